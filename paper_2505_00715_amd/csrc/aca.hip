// Batched ACA of admissible blocks across frequencies, recompression, and the
// per-frequency H-matrix faces (Sec. 4).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "internal.h"
#include "lowrank.h"
#include "near.h"

namespace gcq {

// ---- 2D ACA kernels: one wave per (block, frequency) pair ------------------------
template <typename T, bool ALLFAR, bool DLP>
struct PlainEntry {
  const Tab* tab;
  int rb, cb;
  double sr, si;
  bool all_far;
  __device__ void prep_row(int) {}
  __device__ void prep_col(int) {}
  __device__ cpx<T> part(int i, int j, int p, int P) const {
    return op_entry_part<T, ALLFAR, DLP>(*tab, rb + i, cb + j, sr, si, all_far, p, P);
  }
};

// ALLFAR = true serves the pairs of blocks without self/near-tier entries,
// ALLFAR = false the others; each instance skips the pairs of the other kind.
// NW waves work on one pair together; DLP: entries of the double layer.
template <typename T, bool ALLFAR, int NW, bool DLP>
__global__ void __launch_bounds__(NW * 64) aca_kernel(Tab tab, const PairDesc* __restrict__ pairs,
                                                      const int* __restrict__ order, int npairs,
                                                      unsigned char* __restrict__ ws, double tol,
                                                      int max_rank, int* __restrict__ out_rank,
                                                      int* __restrict__ out_status,
                                                      int* __restrict__ counter) {
  __shared__ AcaShared<T> sm;
  __shared__ int slot;
  const int tid = threadIdx.x;
  for (;;) {
    int idx;
    if constexpr (NW == 1) {
      idx = 0;
      if (tid == 0) idx = atomicAdd(counter, 1);
      idx = __shfl(idx, 0, WAVE);
    } else {
      if (tid == 0) slot = atomicAdd(counter, 1);
      __syncthreads();
      idx = uni(slot);
      __syncthreads();
    }
    if (idx >= npairs) break;
    const int pid = order ? order[idx] : idx;
    const PairDesc d = pairs[pid];
    if ((d.all_far != 0) != ALLFAR) continue;
    cpx<T>* U = reinterpret_cast<cpx<T>*>(ws + d.ws);
    cpx<T>* W = U + int64_t(d.cap) * d.m;
    cpx<double>* GU = reinterpret_cast<cpx<double>*>(ws + d.ws + ws_gram_off<T>(d.cap, d.m, d.n));
    PlainEntry<T, ALLFAR, DLP> ent{&tab, d.rb, d.cb, d.sr, d.si, d.all_far != 0};
    int status = 0;
    const int k = aca_grp<NW, (NW > 1), T>(ent, d.m, d.n, d.cap, max_rank, tol, 0.0, U, W, GU,
                                           GU + d.cap * d.cap, sm, status);
    if (tid == 0) {
      out_rank[pid] = k;
      out_status[pid] = status;
    }
    __syncthreads();
  }
}

template <typename T, bool AF, bool DLP, typename... Args>
static void launch_aca_op(int nw, int grid, hipStream_t st, Args... args) {
  switch (nw) {
    case 1: hipLaunchKernelGGL((aca_kernel<T, AF, 1, DLP>), dim3(grid), dim3(64), 0, st, args...); break;
    case 2: hipLaunchKernelGGL((aca_kernel<T, AF, 2, DLP>), dim3(grid), dim3(128), 0, st, args...); break;
    default: hipLaunchKernelGGL((aca_kernel<T, AF, 4, DLP>), dim3(grid), dim3(256), 0, st, args...); break;
  }
}
template <typename T, bool AF, typename... Args>
static void launch_aca(bool dlp, int nw, int grid, hipStream_t st, Args... args) {
  if (dlp)
    launch_aca_op<T, AF, true>(nw, grid, st, args...);
  else
    launch_aca_op<T, AF, false>(nw, grid, st, args...);
}

// rank classes of the recompression: class c holds the pairs whose ACA rank k
// lies in (RC_LO[c], RC_LO[c + 1]]
constexpr int RC_N = 7;
__constant__ int RC_LO[RC_N + 1] = {-1, 8, 12, 16, 18, 24, 32, 64};
__device__ __forceinline__ int rank_class(int k) {
  int c = 0;
  while (c < RC_N - 1 && k > RC_LO[c + 1]) ++c;
  return c;
}

// the pairs of each class, in one list (class by class): cls[0 .. RC_N) the
// class sizes, cls[RC_N .. 2 RC_N) scatter cursors, cls[2 RC_N .. 3 RC_N)
// the classes' queue heads, all zero on entry; pass 0 counts, pass 1
// scatters (the class offsets are the sums of the sizes before)
__global__ void __launch_bounds__(256) recompress_classify(const int* __restrict__ rank, int nc,
                                                           int* __restrict__ cls, int* __restrict__ list,
                                                           int pass) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = i < nc ? rank_class(rank[i]) : -1;
  const int lane = threadIdx.x & 63;
  for (int q = 0; q < RC_N; ++q) {
    // one atomic per wave and class: the lanes of class q take consecutive slots
    const unsigned long long mask = __ballot(c == q);
    if (mask == 0) continue;
    const int leader = __ffsll(static_cast<long long>(mask)) - 1;
    const int cnt = __popcll(mask);
    int base = 0;
    if (lane == leader) base = atomicAdd(cls + (pass == 0 ? q : RC_N + q), cnt);
    base = __shfl(base, leader, 64);
    if (pass == 1 && c == q) {
      int off = 0;
      for (int r = 0; r < q; ++r) off += cls[r];
      list[off + base + __popcll(mask & ((1ull << lane) - 1ull))] = i;
    }
  }
}

// recompression of the pairs of class `c` (ranks up to MK): groups of NW waves
// take pairs from the class's queue; their working matrices in LDS sized for MK
// terms (GL: in the group's slice of global scratch instead), so that groups
// of small ranks fit many to a compute unit
template <typename T, int MK, int NW, bool GL>
__global__ void __launch_bounds__(NW * 64) recompress_kernel(const PairDesc* __restrict__ pairs,
                                                             unsigned char* __restrict__ ws,
                                                             const int* __restrict__ rank_in,
                                                             int* __restrict__ out_t, double tol,
                                                             int do_recompress, unsigned char* __restrict__ jws,
                                                             int c, int* __restrict__ cls,
                                                             const int* __restrict__ list) {
  __shared__ cpx<double> mats[GL ? 1 : recompress_mats(MK)];
  __shared__ RecompSharedT<MK> rs;
  __shared__ int slot;
  cpx<double>* M = GL ? reinterpret_cast<cpx<double>*>(jws) + int64_t(blockIdx.x) * recompress_mats(MK) : mats;
  int off = 0;
  for (int r = 0; r < c; ++r) off += cls[r];
  const int size = cls[c];
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) slot = atomicAdd(cls + 2 * RC_N + c, 1);
    __syncthreads();
    const int q = uni(slot);
    if (q >= size) break;
    const int pid = list[off + q];
    const int k = rank_in[pid];
    const PairDesc d = pairs[pid];
    const int cap = d.cap;
    cpx<double>* GU = reinterpret_cast<cpx<double>*>(ws + d.ws + ws_gram_off<T>(cap, d.m, d.n));
    const int t = recompress_grp<NW>(k, cap, GU, GU + cap * cap, tol, 0.0, do_recompress != 0, M, rs);
    if (threadIdx.x == 0) out_t[pid] = t;
  }
}

// the recompression of one chunk: a launch per rank class, the classes spread
// over the context stream and the three side streams so that they run
// together (a class of few large pairs takes about one pair's latency, which
// the classes holding most pairs then cover)
constexpr int RECOMP_GL_GRID = 1024;   // groups of the class whose matrices are in global scratch
template <typename T>
static int launch_recompress(gcq_context* ctx, int nc, const PairDesc* pairs, unsigned char* ws,
                             const int* rank, int* t, double tol, int rec, unsigned char* jws, int* cls,
                             int* list) {
  GCQ_TRY(ensure_side_streams(ctx));
  hipStream_t st = ctx->stream;
  const int cg = (nc + 255) / 256;
  hipLaunchKernelGGL(recompress_classify, dim3(cg), dim3(256), 0, st, rank, nc, cls, list, 0);
  hipLaunchKernelGGL(recompress_classify, dim3(cg), dim3(256), 0, st, rank, nc, cls, list, 1);
  GCQ_HIP(hipEventRecord(ctx->evfork, st));
  for (int i = 0; i < 3; ++i) GCQ_HIP(hipStreamWaitEvent(ctx->side[i], ctx->evfork, 0));
  const int g1 = std::min(nc, 5120), g2 = std::min(nc, 2560), g4 = std::min(nc, 1024);
  hipLaunchKernelGGL((recompress_kernel<T, 64, 4, true>), dim3(std::min(nc, RECOMP_GL_GRID)), dim3(256), 0,
                     ctx->side[0], pairs, ws, rank, t, tol, rec, jws, 6, cls, list);
  hipLaunchKernelGGL((recompress_kernel<T, 32, 4, false>), dim3(g4), dim3(256), 0, ctx->side[0], pairs, ws,
                     rank, t, tol, rec, jws, 5, cls, list);
  hipLaunchKernelGGL((recompress_kernel<T, 24, 2, false>), dim3(g2), dim3(128), 0, ctx->side[0], pairs, ws,
                     rank, t, tol, rec, jws, 4, cls, list);
  hipLaunchKernelGGL((recompress_kernel<T, 18, 2, false>), dim3(g2), dim3(128), 0, ctx->side[1], pairs, ws,
                     rank, t, tol, rec, jws, 3, cls, list);
  hipLaunchKernelGGL((recompress_kernel<T, 16, 2, false>), dim3(g2), dim3(128), 0, st, pairs, ws, rank, t, tol,
                     rec, jws, 2, cls, list);
  hipLaunchKernelGGL((recompress_kernel<T, 12, 1, false>), dim3(g1), dim3(64), 0, ctx->side[2], pairs, ws, rank,
                     t, tol, rec, jws, 1, cls, list);
  hipLaunchKernelGGL((recompress_kernel<T, 8, 1, false>), dim3(g1), dim3(64), 0, ctx->side[2], pairs, ws,
                     rank, t, tol, rec, jws, 0, cls, list);
  GCQ_HIP(hipGetLastError());
  for (int i = 0; i < 3; ++i) {
    GCQ_HIP(hipEventRecord(ctx->evjoin[i], ctx->side[i]));
    GCQ_HIP(hipStreamWaitEvent(st, ctx->evjoin[i], 0));
  }
  return GCQ_OK;
}

// Ubar = U CU, Vbar = conj(W) CV into the compact pool; a group of four waves
// per pair, the coefficients staged in LDS when they fit (two call sites, so
// that the LDS one compiles to LDS reads)
constexpr int APPLY_THREADS = 256;
constexpr int APPLY_LDS = 512;   // coefficients of CU (and of CV) held in LDS
template <typename T>
__global__ void __launch_bounds__(APPLY_THREADS) apply_kernel(const PairDesc* __restrict__ pairs, int npairs,
                                                              const unsigned char* __restrict__ ws,
                                                              const int* __restrict__ rank_in,
                                                              const int* __restrict__ tcut,
                                                              const int64_t* __restrict__ out_off,
                                                              cpx<T>* __restrict__ pool) {
  __shared__ cpx<double> cs[2 * APPLY_LDS];
  for (int pid = blockIdx.x; pid < npairs; pid += gridDim.x) {
    const PairDesc d = pairs[pid];
    const int k = rank_in[pid], t = tcut[pid], cap = d.cap, m = d.m, n = d.n;
    if (t == 0) continue;
    const cpx<T>* U = reinterpret_cast<const cpx<T>*>(ws + d.ws);
    const cpx<double>* CU =
        reinterpret_cast<const cpx<double>*>(ws + d.ws + ws_gram_off<T>(cap, m, n));
    cpx<T>* OU = pool + out_off[pid];
    if (k * t <= APPLY_LDS) {
      __syncthreads();   // the previous pair's readers are done
      for (int e = threadIdx.x; e < k * t; e += APPLY_THREADS) {
        cs[e] = CU[e];
        cs[APPLY_LDS + e] = CU[cap * cap + e];
      }
      __syncthreads();
      apply_factors<T>(k, t, m, n, U, U + int64_t(cap) * m, cs, cs + APPLY_LDS, OU, OU + int64_t(t) * m,
                       threadIdx.x, APPLY_THREADS);
    } else {
      apply_factors<T>(k, t, m, n, U, U + int64_t(cap) * m, CU, CU + cap * cap, OU, OU + int64_t(t) * m,
                       threadIdx.x, APPLY_THREADS);
    }
  }
}

__global__ void zero_int(int* p, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// -------------------------------------------------------------------------------------
struct AcaRun {
  std::vector<PairDesc> desc;
  std::vector<int> far_index;   // far block position (0..n_far-1) per pair
  std::vector<int> slot;        // frequency slot per pair
};

template <typename T>
static int run_aca_pairs(gcq_context* ctx, std::vector<PairDesc>& desc, std::vector<int>& order,
                         double tol, int max_rank, bool recompress, std::vector<int>& rank_aca,
                         std::vector<int>& rank_out, std::vector<int>& status,
                         std::vector<int64_t>& out_off, DevBuf& pool, int64_t& pool_used,
                         double& ms_aca, double& ms_rec, double& ms_apply, int64_t budget) {
  hipStream_t st = ctx->stream;
  const int np = int(desc.size());
  rank_aca.assign(np, 0);
  rank_out.assign(np, 0);
  status.assign(np, 0);
  out_off.assign(np, -1);
  const int dev_cus = ctx->cus;
  // chunks in work-list order, each within the workspace budget
  size_t pos = 0;
  const int64_t pool_used0 = pool_used;
  // tile capacity (terms x (m + n)) of the whole list and of the pairs done:
  // the pool grows to the storage per unit of capacity seen so far times the
  // whole list's (the list runs largest first, so a per-pair average of the
  // first chunks would overshoot)
  int64_t cap_total = 0, cap_done = 0;
  for (int q : order) cap_total += int64_t(desc[q].cap) * (desc[q].m + desc[q].n);
  std::vector<int64_t> pend_off;
  while (pos < order.size()) {
    std::vector<int> chunk;
    int64_t wsz = 0;
    while (pos < order.size()) {
      PairDesc& d = desc[order[pos]];
      int64_t b = ws_bytes<T>(d.cap, d.m, d.n);
      if (!chunk.empty() && wsz + b > budget) break;
      d.ws = wsz;
      wsz += b;
      chunk.push_back(order[pos]);
      ++pos;
    }
    const int nc = int(chunk.size());
    for (int q : chunk) cap_done += int64_t(desc[q].cap) * (desc[q].m + desc[q].n);
    std::vector<PairDesc> cd(nc);
    for (int a = 0; a < nc; ++a) cd[a] = desc[chunk[a]];
    GCQ_TRY(ctx->scratchA.ensure(size_t(wsz) + 256));
    GCQ_TRY(upload(ctx->scratchB, cd, st));
    GCQ_TRY(ctx->scratchC.ensure(sizeof(int) * (4 * size_t(nc) + 32)));
    int* d_rank = ctx->scratchC.as<int>();
    int* d_status = d_rank + nc;
    int* d_t = d_status + nc;
    int* d_counter = d_t + nc;
    int* d_cls = d_counter + 8;      // rank classes of the recompression (3 x 7 counters)
    int* d_list = d_counter + 32;    // the pairs class by class
    hipLaunchKernelGGL(zero_int, dim3(1), dim3(64), 0, st, d_counter, 32);
    int nnf = 0;
    for (int a = 0; a < nc; ++a) nnf += cd[a].all_far == 0;
    const int nw = ctx->tune.aca_waves;
    const int grid = std::min(nc, dev_cus * 32 / nw);
    // recompression scratch first: no allocation between the two timed parts
    GCQ_TRY(ctx->scratchD.ensure(size_t(std::min(nc, RECOMP_GL_GRID)) * recompress_mats(64) * 16));
    GCQ_TRY(timed_begin(ctx));
    launch_aca<T, true>(ctx->H.dlp, nw, grid, st, ctx->tab(), (const PairDesc*)ctx->scratchB.as<PairDesc>(),
                        (const int*)nullptr, nc, ctx->scratchA.as<unsigned char>(), tol, max_rank,
                        d_rank, d_status, d_counter);
    if (nnf > 0)
      launch_aca<T, false>(ctx->H.dlp, nw, std::min(grid, nnf), st, ctx->tab(),
                           (const PairDesc*)ctx->scratchB.as<PairDesc>(), (const int*)nullptr, nc,
                           ctx->scratchA.as<unsigned char>(), tol, max_rank, d_rank, d_status,
                           d_counter + 1);
    GCQ_HIP(hipGetLastError());
    // the recompression follows on the device without a host round trip; the
    // split event divides the region between the two
    GCQ_HIP(hipEventRecord(ctx->evm, st));
    // recompression by rank classes; matrices above 32 terms live in global scratch
    GCQ_TRY(launch_recompress<T>(ctx, nc, ctx->scratchB.as<PairDesc>(), ctx->scratchA.as<unsigned char>(), d_rank,
                                 d_t, tol, recompress ? 1 : 0, ctx->scratchD.as<unsigned char>(), d_cls, d_list));
    GCQ_HIP(hipGetLastError());
    {
      double a = 0.0, r = 0.0;
      GCQ_TRY(timed_end_split(ctx, "aca", "recompress", a, r));
      ms_aca += a;
      ms_rec += r;
    }
    std::vector<int> hr(nc), hs(nc), ht(nc);
    GCQ_HIP(hipMemcpy(hr.data(), d_rank, sizeof(int) * nc, hipMemcpyDeviceToHost));
    GCQ_HIP(hipMemcpy(hs.data(), d_status, sizeof(int) * nc, hipMemcpyDeviceToHost));
    GCQ_HIP(hipMemcpy(ht.data(), d_t, sizeof(int) * nc, hipMemcpyDeviceToHost));
    // offsets in the pool (elements), in chunk order; the pool grows by copy
    std::vector<int64_t> off(nc);
    int64_t need = pool_used;
    for (int a = 0; a < nc; ++a) {
      off[a] = need;
      need += int64_t(ht[a]) * (cd[a].m + cd[a].n);
    }
    const size_t esz = sizeof(cpx<T>);
    if (size_t(need) * esz > pool.bytes) {
      // grow to the size the storage per pair so far projects for the whole
      // work list (one copy instead of a cascade; the old and the new pool
      // coexist during the copy)
      const double ratio = double(need - pool_used0) / double(std::max<int64_t>(cap_done, 1));
      const size_t projected = size_t(double(pool_used0) + ratio * double(cap_total) * 1.05);
      DevBuf bigger;
      GCQ_TRY(bigger.ensure(std::max(size_t(need), projected) * esz + 256));
      if (pool_used > 0)
        GCQ_HIP(hipMemcpyAsync(bigger.p, pool.p, size_t(pool_used) * esz,
                               hipMemcpyDeviceToDevice, st));
      GCQ_HIP(hipStreamSynchronize(st));
      std::swap(bigger.p, pool.p);
      std::swap(bigger.bytes, pool.bytes);
    }
    GCQ_TRY(upload(ctx->scratchD, off, st));  // jacobi scratch no longer needed
    GCQ_TRY(timed_begin(ctx));
    hipLaunchKernelGGL(apply_kernel<T>, dim3(std::min(nc, 65536)), dim3(APPLY_THREADS), 0, st,
                       ctx->scratchB.as<PairDesc>(), nc, ctx->scratchA.as<unsigned char>(), d_rank,
                       d_t, ctx->scratchD.as<int64_t>(), pool.as<cpx<T>>());
    GCQ_HIP(hipGetLastError());
    ms_apply += timed_end(ctx, "apply");
    pool_used = need;
    for (int a = 0; a < nc; ++a) {
      rank_aca[chunk[a]] = hr[a];
      status[chunk[a]] = hs[a];
      rank_out[chunk[a]] = ht[a];
      out_off[chunk[a]] = off[a];
    }
  }
  return GCQ_OK;
}

}  // namespace gcq

namespace gcq {
// Stable order of 0..n-1 by key, largest first (ties in index order): LSD
// radix sort of the inverted keys (keys < 2^33), 8 bits per pass.  The work
// list of the ACA has ~1e6 pairs, which a comparison sort orders in ~0.1 s of
// host time.
static std::vector<int> order_desc_stable(const std::vector<uint64_t>& key) {
  const size_t n = key.size();
  uint64_t kmax = 0;
  for (size_t a = 0; a < n; ++a) kmax = std::max(kmax, key[a]);
  int bits = 0;
  while (bits < 33 && (kmax >> bits) != 0) ++bits;
  std::vector<uint64_t> v(n), tmp(n);
  for (size_t a = 0; a < n; ++a) v[a] = ((kmax - key[a]) << 31) | uint64_t(a);   // (inverted key, index)
  for (int sh = 31; sh < 31 + bits; sh += 8) {
    size_t cnt[257] = {0};
    for (size_t a = 0; a < n; ++a) ++cnt[(v[a] >> sh & 255) + 1];
    for (int b = 0; b < 256; ++b) cnt[b + 1] += cnt[b];
    for (size_t a = 0; a < n; ++a) tmp[cnt[v[a] >> sh & 255]++] = v[a];
    v.swap(tmp);
  }
  std::vector<int> order(n);
  for (size_t a = 0; a < n; ++a) order[a] = int(v[a] & ((uint64_t(1) << 31) - 1));
  return order;
}

// dense near-field blocks of every slot: far-tier entries, then self/near-tier ones
template <typename T, bool DLP>
static void launch_near(gcq_context* ctx, dim3 g1, dim3 g2, int nnear, const double2* sig, int nslot,
                        cpx<T>* out, int64_t stride) {
  hipLaunchKernelGGL((near_far_tier<T, DLP>), g1, dim3(256), 0, ctx->stream, ctx->tab(), ctx->d_blk.as<int>(),
                     ctx->d_near_ids.as<int>(), ctx->d_near_off.as<int64_t>(), 0, nnear, int64_t(0), sig, nslot,
                     out, stride);
  hipLaunchKernelGGL((near_sing<T, DLP>), g2, dim3(256), 0, ctx->stream, ctx->tab(), ctx->d_sing.as<SingEntry>(),
                     int64_t(0), ctx->n_sing, int64_t(0), sig, nslot, out, stride);
}

int rank_predict_device(gcq_context* ctx, const float* d_x, int m, float* d_out);
void rank_features_host(gcq_context* ctx, const std::vector<int>& freqs, std::vector<float>& feat);
}  // namespace gcq

using namespace gcq;

extern "C" {

GCQ_API int gcq_aca_blocks(gcq_context* ctx, const int32_t* freq_idx, int32_t n_fidx, double tol,
                           int32_t max_rank, int32_t precision, uint32_t flags,
                           gcq_aca_stats* stats) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!ctx->have_tree || !ctx->have_freq)
    return fail(GCQ_ERR_STATE, "upload mesh, frequencies and build the tree first");
  if (precision != GCQ_C128 && precision != GCQ_C64)
    return fail(GCQ_ERR_ARG, "unknown precision %d", precision);
  if (!(tol >= 0.0) || !std::isfinite(tol)) return fail(GCQ_ERR_ARG, "tol must be >= 0");
  if (max_rank < 1 || max_rank > 64) return fail(GCQ_ERR_ARG, "max_rank must be in 1..64");
  GCQ_HIP(hipSetDevice(ctx->device));
  HFaces& H = ctx->H;
  H.valid = false;
  H.dlp = (flags & GCQ_FLAG_DOUBLE_LAYER) != 0;
  if (H.dlp && (flags & GCQ_FLAG_USE_PREDICTOR))
    return fail(GCQ_ERR_ARG, "the rank model is trained on the single layer; no predictor with the double layer");
  // representatives to approximate
  std::vector<int> fr;
  if (freq_idx && n_fidx > 0) {
    for (int a = 0; a < n_fidx; ++a) {
      int k = freq_idx[a];
      if (k < 0 || k >= ctx->L) return fail(GCQ_ERR_ARG, "frequency index out of range");
      if (ctx->rep[k] != k) return fail(GCQ_ERR_ARG, "frequency %d is not a representative", k);
      fr.push_back(k);
    }
  } else {
    fr = ctx->K;
  }
  const int nslot = int(fr.size());
  const int nfar = int(ctx->far_ids.size());
  H.precision = precision;
  H.freqs = fr;
  H.fslot.assign(ctx->L, -1);
  for (int q = 0; q < nslot; ++q) H.fslot[fr[q]] = q;
  // near field: dense blocks at every frequency slot, [slot][near storage];
  // enqueued first, so that the device evaluates them while the host builds
  // the pair descriptors (own events: the ACA launches below time themselves)
  const int nnear = int(ctx->near_ids.size());
  H.near_off = ctx->near_off;
  const int64_t acc_near = ctx->near_total;
  H.near_slot_elems = acc_near;
  {
    const size_t esz0 = csize(precision);
    GCQ_TRY(H.near.ensure(size_t(acc_near) * nslot * esz0 + 256));
  }
  GCQ_TRY(upload(H.d_near_off, H.near_off, ctx->stream));
  {
    std::vector<double2> sg(nslot);
    for (int q = 0; q < nslot; ++q) {
      std::complex<double> v = ctx->s[fr[q]] / ctx->c;
      sg[q] = make_double2(v.real(), v.imag());
    }
    GCQ_TRY(upload(H.d_sig, sg, ctx->stream));
  }
  struct EventPair {   // destroyed on every return path
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } en;
  GCQ_HIP(hipEventCreate(&en.a));
  GCQ_HIP(hipEventCreate(&en.b));
  GCQ_HIP(hipEventRecord(en.a, ctx->stream));
  if (nnear > 0) {
    const dim3 g1(std::min(nnear, 65536)), g2(4096);
    if (precision == GCQ_C128) {
      if (H.dlp)
        launch_near<double, true>(ctx, g1, g2, nnear, H.d_sig.as<double2>(), nslot, H.near.as<cpx<double>>(), acc_near);
      else
        launch_near<double, false>(ctx, g1, g2, nnear, H.d_sig.as<double2>(), nslot, H.near.as<cpx<double>>(), acc_near);
    } else {
      if (H.dlp)
        launch_near<float, true>(ctx, g1, g2, nnear, H.d_sig.as<double2>(), nslot, H.near.as<cpx<float>>(), acc_near);
      else
        launch_near<float, false>(ctx, g1, g2, nnear, H.d_sig.as<double2>(), nslot, H.near.as<cpx<float>>(), acc_near);
    }
  }
  GCQ_HIP(hipGetLastError());
  GCQ_HIP(hipEventRecord(en.b, ctx->stream));
  // pair descriptors: (far block f, slot q) at index q * nfar + f
  std::vector<PairDesc> desc(size_t(nslot) * nfar);
  for (int q = 0; q < nslot; ++q) {
    std::complex<double> sg = ctx->s[fr[q]] / ctx->c;
    for (int f = 0; f < nfar; ++f) {
      const Block& B = ctx->blocks[ctx->far_ids[f]];
      const Cluster& A = ctx->clusters[B.row];
      const Cluster& C = ctx->clusters[B.col];
      PairDesc& d = desc[size_t(q) * nfar + f];
      d.rb = A.begin;
      d.m = A.end - A.begin;
      d.cb = C.begin;
      d.n = C.end - C.begin;
      if (d.m > ACA_MAXM) return fail(GCQ_ERR_UNSUPPORTED, "block with %d rows exceeds %d", d.m, ACA_MAXM);
      d.all_far = B.all_far ? 1 : 0;
      d.cap = std::min(std::min(d.m, d.n), int(max_rank));
      d.sr = sg.real();
      d.si = sg.imag();
      d.ws = 0;
    }
  }
  std::vector<int> order(desc.size());
  std::iota(order.begin(), order.end(), 0);
  const bool predict = (flags & GCQ_FLAG_USE_PREDICTOR) != 0;
  if (predict) {
    // tile capacities from the rank model: ceil(1.25 r) + 2, multiple of 4,
    // at least 4; work list ordered by predicted cost (largest first)
    if (!ctx->M.trained) return fail(GCQ_ERR_STATE, "train or set the rank model first");
    std::vector<float> feat;
    rank_features_host(ctx, fr, feat);  // [far][slot][5]
    const size_t np = desc.size();
    std::vector<float> xs(np * 5);
    for (int q = 0; q < nslot; ++q)
      for (int f = 0; f < nfar; ++f)
        for (int a = 0; a < 5; ++a)
          xs[(size_t(q) * nfar + f) * 5 + a] =
              (feat[(size_t(f) * nslot + q) * 5 + a] - ctx->M.mean[a]) / ctx->M.stdv[a];
    DevBuf dx, dy;
    GCQ_TRY(upload(dx, xs, ctx->stream));
    GCQ_TRY(dy.ensure(sizeof(float) * np));
    GCQ_TRY(timed_begin(ctx));
    GCQ_TRY(rank_predict_device(ctx, dx.as<float>(), int(np), dy.as<float>()));
    ctx->kernel_ms["predict"] = timed_end(ctx, "predict");
    std::vector<float> pr(np);
    GCQ_HIP(hipMemcpy(pr.data(), dy.p, sizeof(float) * np, hipMemcpyDeviceToHost));
    std::vector<uint64_t> cost(np);
    for (size_t p = 0; p < np; ++p) {
      double r = std::max(0.0, std::expm1(double(pr[p])));
      int capp = int(std::ceil(1.25 * r)) + 2;
      capp = std::max(4, (capp + 3) / 4 * 4);
      desc[p].cap = std::min(desc[p].cap, capp);
      cost[p] = uint64_t(desc[p].cap) * uint64_t(desc[p].m + desc[p].n);
    }
    order = order_desc_stable(cost);
  }
  std::vector<int> rank_aca, rank_out, status;
  std::vector<int64_t> off;
  int64_t pool_used = 0;
  double ms_aca = 0, ms_rec = 0, ms_apply = 0;
  const bool rec = (flags & GCQ_FLAG_RECOMPRESS) != 0;
  const int64_t budget = int64_t(16) << 30;
  int64_t n_overflow_pairs = 0;
  int rc;
  if (flags & GCQ_FLAG_PER_FREQ_LAUNCH) {
    // baseline: one chunk (launch sequence) per frequency, natural order
    rank_aca.assign(desc.size(), 0);
    rank_out.assign(desc.size(), 0);
    status.assign(desc.size(), 0);
    off.assign(desc.size(), 0);
    for (int q = 0; q < nslot; ++q) {
      std::vector<PairDesc> dq(desc.begin() + size_t(q) * nfar, desc.begin() + size_t(q + 1) * nfar);
      std::vector<int> oq(nfar);
      std::iota(oq.begin(), oq.end(), 0);
      std::vector<int> ra, ro, stt;
      std::vector<int64_t> of;
      rc = precision == GCQ_C128
               ? run_aca_pairs<double>(ctx, dq, oq, tol, max_rank, rec, ra, ro, stt, of, H.factors,
                                       pool_used, ms_aca, ms_rec, ms_apply, budget)
               : run_aca_pairs<float>(ctx, dq, oq, tol, max_rank, rec, ra, ro, stt, of, H.factors,
                                      pool_used, ms_aca, ms_rec, ms_apply, budget);
      if (rc < 0) return rc;
      for (int f = 0; f < nfar; ++f) {
        rank_aca[size_t(q) * nfar + f] = ra[f];
        rank_out[size_t(q) * nfar + f] = ro[f];
        status[size_t(q) * nfar + f] = stt[f];
        off[size_t(q) * nfar + f] = of[f];
      }
    }
  } else {
    rc = precision == GCQ_C128
             ? run_aca_pairs<double>(ctx, desc, order, tol, max_rank, rec, rank_aca, rank_out,
                                     status, off, H.factors, pool_used, ms_aca, ms_rec, ms_apply,
                                     budget)
             : run_aca_pairs<float>(ctx, desc, order, tol, max_rank, rec, rank_aca, rank_out,
                                    status, off, H.factors, pool_used, ms_aca, ms_rec, ms_apply,
                                    budget);
    if (rc < 0) return rc;
    if (predict) {
      // pairs whose tile was too small run again at full capacity; the
      // adaptive ACA decides the rank
      std::vector<PairDesc> od;
      std::vector<int> who;
      for (size_t p = 0; p < desc.size(); ++p)
        if (status[p] & ST_OVERFLOW) {
          PairDesc d = desc[p];
          d.cap = std::min(std::min(d.m, d.n), int(max_rank));
          od.push_back(d);
          who.push_back(int(p));
        }
      n_overflow_pairs = int64_t(who.size());
      if (!od.empty()) {
        std::vector<int> oo(od.size());
        std::iota(oo.begin(), oo.end(), 0);
        std::vector<int> ra, ro, stt;
        std::vector<int64_t> of;
        rc = precision == GCQ_C128
                 ? run_aca_pairs<double>(ctx, od, oo, tol, max_rank, rec, ra, ro, stt, of,
                                         H.factors, pool_used, ms_aca, ms_rec, ms_apply, budget)
                 : run_aca_pairs<float>(ctx, od, oo, tol, max_rank, rec, ra, ro, stt, of,
                                        H.factors, pool_used, ms_aca, ms_rec, ms_apply, budget);
        if (rc < 0) return rc;
        for (size_t a = 0; a < who.size(); ++a) {
          rank_aca[who[a]] = ra[a];
          rank_out[who[a]] = ro[a];
          status[who[a]] = stt[a];
          off[who[a]] = of[a];
        }
      }
    }
  }
  // near field, launched above
  const int64_t acc = ctx->near_total;
  const size_t esz = csize(precision);
  // per (far block, slot) tables in [slot][far] order
  H.off = off;
  H.rank = rank_out;
  GCQ_TRY(upload(H.d_off, H.off, ctx->stream));
  GCQ_TRY(upload(H.d_rank, H.rank, ctx->stream));
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  float ms_near_f = 0.f;
  GCQ_HIP(hipEventElapsedTime(&ms_near_f, en.a, en.b));
  const double ms_near = ms_near_f;
  ctx->kernel_ms["near"] = ms_near;
  H.storage_bytes = int64_t(esz) * (pool_used + acc * nslot);
  H.valid = true;
  ctx->kernel_ms["aca_blocks"] = ms_aca + ms_rec + ms_apply + ms_near;
  ctx->kernel_ms["aca_total"] = ms_aca;
  ctx->kernel_ms["recompress_total"] = ms_rec;
  ctx->kernel_ms["apply_total"] = ms_apply;
  int ncap = 0, rmax = 0;
  int64_t rsum = 0, rasum = 0, nover = 0, ents = 0;
  for (size_t p = 0; p < desc.size(); ++p) {
    ncap += (status[p] & ST_CAPPED) != 0;
    (void)nover;
    rmax = std::max(rmax, rank_out[p]);
    rsum += rank_out[p];
    rasum += rank_aca[p];
    ents += int64_t(rank_aca[p]) * (desc[p].m + desc[p].n);
  }
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->n_pairs = int64_t(desc.size());
    stats->aca_rank_sum = rasum;
    stats->rank_sum = rsum;
    stats->rank_max = rmax;
    stats->n_capped = ncap;
    stats->n_overflow = n_overflow_pairs;
    stats->entries = ents;
    stats->storage_bytes = H.storage_bytes;
    stats->device_ms = ms_aca + ms_rec + ms_apply;
  }
  return ncap > 0 ? GCQ_RANK_CAPPED : GCQ_OK;
}

GCQ_API int gcq_aca_ranks(gcq_context* ctx, int32_t* ranks, int64_t n) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!ctx->H.valid) return fail(GCQ_ERR_STATE, "run gcq_aca_blocks first");
  const int64_t nfar = int64_t(ctx->far_ids.size()), nslot = int64_t(ctx->H.freqs.size());
  if (!ranks || n != nfar * nslot) return fail(GCQ_ERR_ARG, "ranks must hold %lld values", (long long)(nfar * nslot));
  for (int64_t q = 0; q < nslot; ++q)
    for (int64_t f = 0; f < nfar; ++f) ranks[f * nslot + q] = ctx->H.rank[q * nfar + f];
  return GCQ_OK;
}

GCQ_API int gcq_get_block_factors(gcq_context* ctx, int32_t block, int32_t freq, gcq_c128* U,
                                  gcq_c128* V, int32_t cap, int32_t* rank) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!ctx->H.valid) return fail(GCQ_ERR_STATE, "run gcq_aca_blocks first");
  if (block < 0 || block >= int(ctx->blocks.size()) || !ctx->blocks[block].admissible)
    return fail(GCQ_ERR_ARG, "block %d is not an admissible block", block);
  if (freq < 0 || freq >= ctx->L || ctx->H.fslot[freq] < 0)
    return fail(GCQ_ERR_ARG, "frequency %d was not approximated", freq);
  if (!U || !V || !rank) return fail(GCQ_ERR_ARG, "NULL output");
  const int f = int(std::lower_bound(ctx->far_ids.begin(), ctx->far_ids.end(), block) -
                    ctx->far_ids.begin());
  const size_t pi = size_t(ctx->H.fslot[freq]) * ctx->far_ids.size() + f;
  const int r = ctx->H.rank[pi];
  *rank = r;
  if (r > cap) return fail(GCQ_ERR_ARG, "rank %d exceeds cap %d", r, cap);
  const Block& B = ctx->blocks[block];
  const int m = ctx->clusters[B.row].end - ctx->clusters[B.row].begin;
  const int n = ctx->clusters[B.col].end - ctx->clusters[B.col].begin;
  const int64_t cnt = int64_t(r) * (m + n);
  if (cnt == 0) return GCQ_OK;
  std::vector<gcq_c128> tmp(cnt);
  if (ctx->H.precision == GCQ_C128) {
    GCQ_HIP(hipMemcpy(tmp.data(), ctx->H.factors.as<cpx<double>>() + ctx->H.off[pi],
                      cnt * sizeof(gcq_c128), hipMemcpyDeviceToHost));
  } else {
    std::vector<cpx<float>> t32(cnt);
    GCQ_HIP(hipMemcpy(t32.data(), ctx->H.factors.as<cpx<float>>() + ctx->H.off[pi],
                      cnt * sizeof(cpx<float>), hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < cnt; ++e) tmp[e] = {t32[e].re, t32[e].im};
  }
  std::memcpy(U, tmp.data(), sizeof(gcq_c128) * int64_t(r) * m);
  std::memcpy(V, tmp.data() + int64_t(r) * m, sizeof(gcq_c128) * int64_t(r) * n);
  return GCQ_OK;
}

}  // extern "C"
