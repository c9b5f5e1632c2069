// Rank-prediction network: 5 -> 64 -> 64 -> 1 with tanh hidden layers, in
// float, trained on the GPU with the library's own forward, backward and Adam
// kernels.  Parameter layout W1(64x5) b1(64) W2(64x64) b2(64) W3(1x64) b3(1),
// row-major.  Loss 1/2 mean (y - t)^2 on targets log(1 + rank).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <random>

#include "internal.h"

namespace gcq {

constexpr int NIN = 5, NH = 64;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NH, NPARAM = OB3 + 1;
static_assert(NPARAM == 4609, "parameter count");

// forward: one thread per sample; weights staged in LDS.  H1, H2 (B x 64) are
// kept for the backward pass when non-null.
__global__ void __launch_bounds__(256) mlp_forward(const float* __restrict__ P,
                                                   const float* __restrict__ X,
                                                   const int* __restrict__ idx, int B,
                                                   float* __restrict__ H1, float* __restrict__ H2,
                                                   float* __restrict__ Y) {
  __shared__ float w[NPARAM];
  for (int e = threadIdx.x; e < NPARAM; e += blockDim.x) w[e] = P[e];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const int row = idx ? idx[s] : s;
  float x[NIN];
#pragma unroll
  for (int a = 0; a < NIN; ++a) x[a] = X[int64_t(row) * NIN + a];
  float h1[NH];
#pragma unroll
  for (int o = 0; o < NH; ++o) {
    float acc = w[OB1 + o];
#pragma unroll
    for (int a = 0; a < NIN; ++a) acc += w[OW1 + o * NIN + a] * x[a];
    h1[o] = tanhf(acc);
    if (H1) H1[int64_t(s) * NH + o] = h1[o];
  }
  float y = w[OB3];
  for (int o = 0; o < NH; ++o) {
    float acc = w[OB2 + o];
#pragma unroll
    for (int a = 0; a < NH; ++a) acc += w[OW2 + o * NH + a] * h1[a];
    const float h2 = tanhf(acc);
    if (H2) H2[int64_t(s) * NH + o] = h2;
    y += w[OW3 + o] * h2;
  }
  Y[s] = y;
}

// backward through the activations: E = (y - t) / B, D2 = E W3 (1 - H2^2),
// D1 = (D2 W2) (1 - H1^2); one thread per sample
__global__ void __launch_bounds__(256) mlp_backward_act(const float* __restrict__ P,
                                                        const float* __restrict__ T,
                                                        const int* __restrict__ idx, int B,
                                                        const float* __restrict__ Y,
                                                        const float* __restrict__ H1,
                                                        const float* __restrict__ H2,
                                                        float* __restrict__ E,
                                                        float* __restrict__ D1,
                                                        float* __restrict__ D2) {
  __shared__ float w[NPARAM];
  for (int e = threadIdx.x; e < NPARAM; e += blockDim.x) w[e] = P[e];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  const int row = idx ? idx[s] : s;
  const float e = (Y[s] - T[row]) / float(B);
  E[s] = e;
  float d2[NH];
#pragma unroll
  for (int o = 0; o < NH; ++o) {
    const float h = H2[int64_t(s) * NH + o];
    d2[o] = e * w[OW3 + o] * (1.f - h * h);
    D2[int64_t(s) * NH + o] = d2[o];
  }
  for (int a = 0; a < NH; ++a) {
    float acc = 0.f;
#pragma unroll
    for (int o = 0; o < NH; ++o) acc += d2[o] * w[OW2 + o * NH + a];
    const float h = H1[int64_t(s) * NH + a];
    D1[int64_t(s) * NH + a] = acc * (1.f - h * h);
  }
}

// parameter gradients: one thread per parameter, summing over the batch
__global__ void __launch_bounds__(256) mlp_grad(const float* __restrict__ X,
                                                const int* __restrict__ idx, int B,
                                                const float* __restrict__ H1,
                                                const float* __restrict__ H2,
                                                const float* __restrict__ E,
                                                const float* __restrict__ D1,
                                                const float* __restrict__ D2,
                                                float* __restrict__ G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  float acc = 0.f;
  if (p < OB1) {  // W1[o][a] = sum_s D1[s][o] X[s][a]
    const int o = p / NIN, a = p % NIN;
    for (int s = 0; s < B; ++s) acc += D1[int64_t(s) * NH + o] * X[int64_t(idx ? idx[s] : s) * NIN + a];
  } else if (p < OW2) {
    const int o = p - OB1;
    for (int s = 0; s < B; ++s) acc += D1[int64_t(s) * NH + o];
  } else if (p < OB2) {  // W2[o][a] = sum_s D2[s][o] H1[s][a]
    const int o = (p - OW2) / NH, a = (p - OW2) % NH;
    for (int s = 0; s < B; ++s) acc += D2[int64_t(s) * NH + o] * H1[int64_t(s) * NH + a];
  } else if (p < OW3) {
    const int o = p - OB2;
    for (int s = 0; s < B; ++s) acc += D2[int64_t(s) * NH + o];
  } else if (p < OB3) {  // W3[0][a] = sum_s E[s] H2[s][a]
    const int a = p - OW3;
    for (int s = 0; s < B; ++s) acc += E[s] * H2[int64_t(s) * NH + a];
  } else {
    for (int s = 0; s < B; ++s) acc += E[s];
  }
  G[p] = acc;
}

// Adam with bias correction (step counts from 1)
__global__ void mlp_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                         float* __restrict__ V, int step, float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NPARAM) return;
  const float g = G[p];
  const float m = b1 * M[p] + (1.f - b1) * g;
  const float v = b2 * V[p] + (1.f - b2) * g * g;
  M[p] = m;
  V[p] = v;
  const float mh = m / (1.f - powf(b1, float(step)));
  const float vh = v / (1.f - powf(b2, float(step)));
  P[p] -= lr * mh / (sqrtf(vh) + eps);
}

// loss partial sums: 1/2 sum (y - t)^2 per block
__global__ void __launch_bounds__(256) mlp_loss(const float* __restrict__ Y,
                                                const float* __restrict__ T,
                                                const int* __restrict__ idx, int B,
                                                float* __restrict__ out) {
  __shared__ float sh[4];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  float v = 0.f;
  if (s < B) {
    const float d = Y[s] - T[idx ? idx[s] : s];
    v = 0.5f * d * d;
  }
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

static void glorot(std::vector<float>& p, uint64_t seed) {
  std::mt19937_64 rng(seed);
  p.assign(NPARAM, 0.f);
  auto fill = [&](int off, int fo, int fi) {
    const double lim = std::sqrt(6.0 / (fo + fi));
    std::uniform_real_distribution<double> u(-lim, lim);
    for (int e = 0; e < fo * fi; ++e) p[off + e] = float(u(rng));
  };
  fill(OW1, NH, NIN);
  fill(OW2, NH, NH);
  fill(OW3, 1, NH);
}

struct MlpBufs {
  DevBuf x, t, idx, h1, h2, e, d1, d2, y, g, m, v, loss;
  int cap = 0;
  int ensure(int B) {
    if (B <= cap) return GCQ_OK;
    GCQ_TRY(h1.ensure(sizeof(float) * size_t(B) * NH));
    GCQ_TRY(h2.ensure(sizeof(float) * size_t(B) * NH));
    GCQ_TRY(d1.ensure(sizeof(float) * size_t(B) * NH));
    GCQ_TRY(d2.ensure(sizeof(float) * size_t(B) * NH));
    GCQ_TRY(e.ensure(sizeof(float) * size_t(B)));
    GCQ_TRY(y.ensure(sizeof(float) * size_t(B)));
    GCQ_TRY(loss.ensure(sizeof(float) * size_t(B / 256 + 2)));
    cap = B;
    return GCQ_OK;
  }
};

// loss and gradient of one batch (rows idx[0..B) of the uploaded set) into bufs.g
static int fwd_bwd(gcq_context* ctx, MlpBufs& b, const float* P, const int* idx, int B,
                   float* loss_out) {
  hipStream_t st = ctx->stream;
  const int nb = (B + 255) / 256;
  hipLaunchKernelGGL(mlp_forward, dim3(nb), dim3(256), 0, st, P, b.x.as<float>(), idx, B,
                     b.h1.as<float>(), b.h2.as<float>(), b.y.as<float>());
  hipLaunchKernelGGL(mlp_backward_act, dim3(nb), dim3(256), 0, st, P, b.t.as<float>(), idx, B,
                     b.y.as<float>(), b.h1.as<float>(), b.h2.as<float>(), b.e.as<float>(),
                     b.d1.as<float>(), b.d2.as<float>());
  hipLaunchKernelGGL(mlp_grad, dim3((NPARAM + 255) / 256), dim3(256), 0, st, b.x.as<float>(), idx,
                     B, b.h1.as<float>(), b.h2.as<float>(), b.e.as<float>(), b.d1.as<float>(),
                     b.d2.as<float>(), b.g.as<float>());
  if (loss_out) {
    hipLaunchKernelGGL(mlp_loss, dim3(nb), dim3(256), 0, st, b.y.as<float>(), b.t.as<float>(), idx,
                       B, b.loss.as<float>());
    std::vector<float> part(nb);
    GCQ_HIP(hipMemcpyAsync(part.data(), b.loss.p, sizeof(float) * nb, hipMemcpyDeviceToHost, st));
    GCQ_HIP(hipStreamSynchronize(st));
    double s = 0;
    for (float v : part) s += v;
    *loss_out = float(s / B);
  }
  return GCQ_OK;
}

static int ensure_params(gcq_context* ctx) {
  RankModel& M = ctx->M;
  if (M.params.empty()) glorot(M.params, 0);
  GCQ_TRY(upload(M.d_params, M.params, ctx->stream));
  return GCQ_OK;
}

// prediction of log(1 + rank) for m standardised rows already on the device
int rank_predict_device(gcq_context* ctx, const float* d_x, int m, float* d_out) {
  GCQ_TRY(ensure_params(ctx));
  hipLaunchKernelGGL(mlp_forward, dim3((m + 255) / 256), dim3(256), 0, ctx->stream,
                     ctx->M.d_params.as<float>(), d_x, (const int*)nullptr, m, (float*)nullptr,
                     (float*)nullptr, d_out);
  GCQ_HIP(hipGetLastError());
  return GCQ_OK;
}

void rank_features_host(gcq_context* ctx, const std::vector<int>& freqs, std::vector<float>& feat) {
  const int nfar = int(ctx->far_ids.size());
  feat.assign(size_t(nfar) * freqs.size() * 5, 0.f);
  // per frequency |s|, Re s, |Im s| (the same expressions as per pair)
  std::vector<double> sabs(freqs.size()), sre(freqs.size()), sim(freqs.size());
  for (size_t q = 0; q < freqs.size(); ++q) {
    const std::complex<double> s = ctx->s[freqs[q]];
    sabs[q] = std::abs(s);
    sre[q] = s.real();
    sim[q] = std::abs(s.imag());
  }
  for (int f = 0; f < nfar; ++f) {
    const Block& B = ctx->blocks[ctx->far_ids[f]];
    const Cluster& A = ctx->clusters[B.row];
    const Cluster& C = ctx->clusters[B.col];
    auto diam = [](const Cluster& c) {
      double dx = c.bmax[0] - c.bmin[0], dy = c.bmax[1] - c.bmin[1], dz = c.bmax[2] - c.bmin[2];
      return std::sqrt(dx * dx + dy * dy + dz * dz);
    };
    double g[3];
    for (int k = 0; k < 3; ++k)
      g[k] = std::max(0.0, std::max(A.bmin[k] - C.bmax[k], C.bmin[k] - A.bmax[k]));
    const double dist = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    const double dm = std::max(diam(A), diam(C));
    const float lm = float(std::log2(double(A.end - A.begin)));
    const float ln = float(std::log2(double(C.end - C.begin)));
    for (size_t q = 0; q < freqs.size(); ++q) {
      float* o = &feat[(size_t(f) * freqs.size() + q) * 5];
      o[0] = float(dm * sabs[q] / ctx->c);
      o[1] = float(dist * sre[q] / ctx->c);
      o[2] = float(dist * sim[q] / ctx->c);
      o[3] = lm;
      o[4] = ln;
    }
  }
}

}  // namespace gcq

using namespace gcq;

extern "C" {

GCQ_API int gcq_rank_features(gcq_context* ctx, const int32_t* freq_idx, int32_t n_fidx,
                              float* feat) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!ctx->have_tree || !ctx->have_freq) return fail(GCQ_ERR_STATE, "build the tree first");
  if (!freq_idx || n_fidx < 0 || !feat) return fail(GCQ_ERR_ARG, "bad arguments");
  std::vector<int> fr(freq_idx, freq_idx + n_fidx);
  for (int k : fr)
    if (k < 0 || k >= ctx->L) return fail(GCQ_ERR_ARG, "frequency index out of range");
  std::vector<float> f;
  rank_features_host(ctx, fr, f);
  std::memcpy(feat, f.data(), sizeof(float) * f.size());
  return GCQ_OK;
}

GCQ_API int gcq_rank_model_train(gcq_context* ctx, const float* feat, const float* target,
                                 int64_t m, const gcq_train_cfg* cfg, gcq_train_stats* stats) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!feat || !target || m < 1 || !cfg) return fail(GCQ_ERR_ARG, "bad arguments");
  if (cfg->epochs < 1 || cfg->batch < 1 || !(cfg->lr > 0.f))
    return fail(GCQ_ERR_ARG, "bad training configuration");
  GCQ_HIP(hipSetDevice(ctx->device));
  RankModel& M = ctx->M;
  // standardisation fitted on the training set
  for (int a = 0; a < NIN; ++a) {
    double mu = 0, sd = 0;
    for (int64_t s = 0; s < m; ++s) mu += feat[s * NIN + a];
    mu /= double(m);
    for (int64_t s = 0; s < m; ++s) sd += (feat[s * NIN + a] - mu) * (feat[s * NIN + a] - mu);
    sd = std::sqrt(sd / double(m));
    M.mean[a] = float(mu);
    M.stdv[a] = float(sd > 1e-12 ? sd : 1.0);
  }
  std::vector<float> xs(size_t(m) * NIN);
  for (int64_t s = 0; s < m; ++s)
    for (int a = 0; a < NIN; ++a) xs[s * NIN + a] = (feat[s * NIN + a] - M.mean[a]) / M.stdv[a];
  std::vector<float> ts(target, target + m);
  glorot(M.params, cfg->seed);
  GCQ_TRY(upload(M.d_params, M.params, ctx->stream));
  MlpBufs b;
  const int B = int(std::min<int64_t>(cfg->batch, m));
  GCQ_TRY(b.ensure(B));
  GCQ_TRY(upload(b.x, xs, ctx->stream));
  GCQ_TRY(upload(b.t, ts, ctx->stream));
  GCQ_TRY(b.g.ensure(sizeof(float) * NPARAM));
  std::vector<float> zeros(NPARAM, 0.f);
  GCQ_TRY(upload(b.m, zeros, ctx->stream));
  GCQ_TRY(upload(b.v, zeros, ctx->stream));
  std::vector<int> perm(m);
  std::iota(perm.begin(), perm.end(), 0);
  std::mt19937_64 rng(cfg->seed ^ 0x9e3779b97f4a7c15ull);
  GCQ_TRY(b.idx.ensure(sizeof(int) * size_t(m)));
  int step = 0;
  float lfirst = 0, llast = 0;
  GCQ_TRY(timed_begin(ctx));
  for (int ep = 0; ep < cfg->epochs; ++ep) {
    std::shuffle(perm.begin(), perm.end(), rng);
    GCQ_HIP(hipMemcpyAsync(b.idx.p, perm.data(), sizeof(int) * m, hipMemcpyHostToDevice, ctx->stream));
    double lsum = 0;
    int nbatch = 0;
    for (int64_t o = 0; o + B <= m || (o < m && nbatch == 0); o += B) {
      const int bb = int(std::min<int64_t>(B, m - o));
      float l = 0;
      const bool want = (ep == 0 || ep == cfg->epochs - 1);
      GCQ_TRY(fwd_bwd(ctx, b, M.d_params.as<float>(), b.idx.as<int>() + o, bb, want ? &l : nullptr));
      ++step;
      hipLaunchKernelGGL(mlp_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, ctx->stream,
                         M.d_params.as<float>(), b.g.as<float>(), b.m.as<float>(), b.v.as<float>(),
                         step, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps);
      lsum += l;
      ++nbatch;
    }
    if (ep == 0) lfirst = float(lsum / nbatch);
    if (ep == cfg->epochs - 1) llast = float(lsum / nbatch);
  }
  GCQ_HIP(hipGetLastError());
  const double ms = timed_end(ctx, "mlp_train");
  GCQ_HIP(hipMemcpy(M.params.data(), M.d_params.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
  M.trained = true;
  if (stats) {
    stats->loss_first = lfirst;
    stats->loss_last = llast;
    stats->device_ms = ms;
  }
  return GCQ_OK;
}

GCQ_API int gcq_rank_model_grad(gcq_context* ctx, const float* feat_std, const float* target,
                                int64_t m, float* loss, float* grad) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!feat_std || !target || m < 1 || m > (1 << 24) || !loss || !grad)
    return fail(GCQ_ERR_ARG, "bad arguments");
  GCQ_HIP(hipSetDevice(ctx->device));
  GCQ_TRY(ensure_params(ctx));
  MlpBufs b;
  GCQ_TRY(b.ensure(int(m)));
  std::vector<float> xs(feat_std, feat_std + m * NIN), ts(target, target + m);
  GCQ_TRY(upload(b.x, xs, ctx->stream));
  GCQ_TRY(upload(b.t, ts, ctx->stream));
  GCQ_TRY(b.g.ensure(sizeof(float) * NPARAM));
  GCQ_TRY(fwd_bwd(ctx, b, ctx->M.d_params.as<float>(), nullptr, int(m), loss));
  GCQ_HIP(hipMemcpy(grad, b.g.p, sizeof(float) * NPARAM, hipMemcpyDeviceToHost));
  return GCQ_OK;
}

GCQ_API int gcq_rank_model_predict(gcq_context* ctx, const float* feat, int64_t m, float* out) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!feat || !out || m < 0) return fail(GCQ_ERR_ARG, "bad arguments");
  if (m == 0) return GCQ_OK;
  GCQ_HIP(hipSetDevice(ctx->device));
  std::vector<float> xs(size_t(m) * NIN);
  for (int64_t s = 0; s < m; ++s)
    for (int a = 0; a < NIN; ++a)
      xs[s * NIN + a] = (feat[s * NIN + a] - ctx->M.mean[a]) / ctx->M.stdv[a];
  DevBuf dx, dy;
  GCQ_TRY(upload(dx, xs, ctx->stream));
  GCQ_TRY(dy.ensure(sizeof(float) * size_t(m)));
  GCQ_TRY(rank_predict_device(ctx, dx.as<float>(), int(m), dy.as<float>()));
  GCQ_HIP(hipMemcpyAsync(out, dy.p, sizeof(float) * m, hipMemcpyDeviceToHost, ctx->stream));
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  return GCQ_OK;
}

GCQ_API int gcq_rank_model_get(gcq_context* ctx, float* params, float* mean, float* stdv) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (ctx->M.params.empty()) glorot(ctx->M.params, 0);
  if (params) std::memcpy(params, ctx->M.params.data(), sizeof(float) * NPARAM);
  if (mean) std::memcpy(mean, ctx->M.mean, sizeof(float) * NIN);
  if (stdv) std::memcpy(stdv, ctx->M.stdv, sizeof(float) * NIN);
  return GCQ_OK;
}

GCQ_API int gcq_rank_model_set(gcq_context* ctx, const float* params, const float* mean,
                               const float* stdv) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!params) return fail(GCQ_ERR_ARG, "params is NULL");
  ctx->M.params.assign(params, params + NPARAM);
  if (mean) std::memcpy(ctx->M.mean, mean, sizeof(float) * NIN);
  if (stdv)
    for (int a = 0; a < NIN; ++a) {
      if (!(stdv[a] > 0.f)) return fail(GCQ_ERR_ARG, "std must be positive");
      ctx->M.stdv[a] = stdv[a];
    }
  ctx->M.trained = true;
  if (ctx->device >= 0) {
    GCQ_HIP(hipSetDevice(ctx->device));
    GCQ_TRY(upload(ctx->M.d_params, ctx->M.params, ctx->stream));
    GCQ_HIP(hipStreamSynchronize(ctx->stream));
  }
  return GCQ_OK;
}

}  // extern "C"
