// Context, mesh and frequency upload, cluster/block tree, dense entries.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <unordered_map>
#include <numeric>

#include "internal.h"
#include "near.h"

namespace gcq {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}

int fail(int code, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int check_device_ptr(gcq_context* ctx, const void* p, const char* what) {
  if (!p) return fail(GCQ_ERR_ARG, "%s is NULL", what);
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(GCQ_ERR_ARG, "%s is not a device pointer", what);
  }
  if (a.type != hipMemoryTypeDevice && a.type != hipMemoryTypeManaged)
    return fail(GCQ_ERR_ARG, "%s is not device memory", what);
  if (a.device != ctx->device)
    return fail(GCQ_ERR_ARG, "%s lives on device %d, the context on %d", what, a.device,
                ctx->device);
  return GCQ_OK;
}

int timed_begin(gcq_context* ctx) {
  GCQ_HIP(hipEventRecord(ctx->ev0, ctx->stream));
  return GCQ_OK;
}

double timed_end(gcq_context* ctx, const char* name) {
  float ms = -1.f;
  if (hipEventRecord(ctx->ev1, ctx->stream) != hipSuccess) return -1.0;
  if (hipEventSynchronize(ctx->ev1) != hipSuccess) return -1.0;
  if (hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1) != hipSuccess) return -1.0;
  ctx->kernel_ms[name] = ms;
  return ms;
}

int timed_end_split(gcq_context* ctx, const char* first, const char* second, double& ms_first,
                    double& ms_second) {
  float a = -1.f, b = -1.f;
  GCQ_HIP(hipEventRecord(ctx->ev1, ctx->stream));
  GCQ_HIP(hipEventSynchronize(ctx->ev1));
  GCQ_HIP(hipEventElapsedTime(&a, ctx->ev0, ctx->evm));
  GCQ_HIP(hipEventElapsedTime(&b, ctx->evm, ctx->ev1));
  ctx->kernel_ms[first] = a;
  ctx->kernel_ms[second] = b;
  ms_first = a;
  ms_second = b;
  return GCQ_OK;
}

// ---- constant tables ------------------------------------------------------------
// 7-point degree-5 rule on the triangle (Radon): centroid and two orbits of 3.
void radon7(double b[7][3], double w[7]) {
  const double sq = std::sqrt(15.0);
  const double a = (6.0 - sq) / 21.0, bb = (6.0 + sq) / 21.0;
  const double wa = (155.0 - sq) / 1200.0, wb = (155.0 + sq) / 1200.0;
  const double pts[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {a, a, 1 - 2 * a}, {a, 1 - 2 * a, a},
                            {1 - 2 * a, a, a},           {bb, bb, 1 - 2 * bb},
                            {bb, 1 - 2 * bb, bb},        {1 - 2 * bb, bb, bb}};
  for (int i = 0; i < 7; ++i) {
    for (int k = 0; k < 3; ++k) b[i][k] = pts[i][k];
    w[i] = i == 0 ? 9.0 / 40.0 : (i < 4 ? wa : wb);
  }
}

// n-point Gauss-Legendre on [0, 1] by Newton iteration on P_n
static void gauss_legendre01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    // ascending order on [0, 1]
    x[n - 1 - i] = 0.5 * (z + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // = (2 / ((1-z^2) P'^2)) / 2
  }
}

static void build_consts(Consts& K) {
  gauss_legendre01(NGL, K.gl_x, K.gl_w);
  double b[7][3], w[7];
  radon7(b, w);
  // two levels of 4-fold midpoint subdivision of the barycentric triangle
  struct Tri { double v[3][3]; };
  std::vector<Tri> tris(1);
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 3; ++k) tris[0].v[a][k] = (a == k) ? 1.0 : 0.0;
  for (int lev = 0; lev < 2; ++lev) {
    std::vector<Tri> nxt;
    for (const Tri& t : tris) {
      double m[3][3];  // ab, bc, ca
      for (int k = 0; k < 3; ++k) {
        m[0][k] = 0.5 * (t.v[0][k] + t.v[1][k]);
        m[1][k] = 0.5 * (t.v[1][k] + t.v[2][k]);
        m[2][k] = 0.5 * (t.v[2][k] + t.v[0][k]);
      }
      const double* kids[4][3] = {{t.v[0], m[0], m[2]}, {m[0], t.v[1], m[1]},
                                  {m[2], m[1], t.v[2]}, {m[0], m[1], m[2]}};
      for (auto& kd : kids) {
        Tri c;
        for (int a = 0; a < 3; ++a)
          for (int k = 0; k < 3; ++k) c.v[a][k] = kd[a][k];
        nxt.push_back(c);
      }
    }
    tris.swap(nxt);
  }
  int q = 0;
  for (const Tri& t : tris)
    for (int i = 0; i < 7; ++i, ++q) {
      for (int k = 0; k < 3; ++k)
        K.nb[q][k] = b[i][0] * t.v[0][k] + b[i][1] * t.v[1][k] + b[i][2] * t.v[2][k];
      K.nw[q] = w[i] / 16.0;
    }
}

}  // namespace gcq

using namespace gcq;

// =====================================================================================
// The tree's derived state, shared by gcq_build_cluster_tree and
// gcq_upload_cluster_tree: inverse permutation, far/near block lists, depth,
// statistics, and on a device context the panel tables in cluster order, the
// block table and the near field's entry lists.  ctx->perm, ctx->clusters
// (ranges, sons, boxes, depths) and ctx->blocks (admissible, all_far) are set.
static int finish_tree(gcq_context* ctx, gcq_tree_info* info) {
#pragma clang fp contract(off)
  const int n = ctx->n;
  const std::vector<double>& cen = ctx->cen;
  const std::vector<double>& vert = ctx->vert;
  ctx->iperm.assign(n, 0);
  for (int p = 0; p < n; ++p) ctx->iperm[ctx->perm[p]] = p;
  ctx->far_ids.clear();
  ctx->near_ids.clear();
  for (size_t b = 0; b < ctx->blocks.size(); ++b)
    (ctx->blocks[b].admissible ? ctx->far_ids : ctx->near_ids).push_back(int(b));
  ctx->depth = 0;
  for (auto& c : ctx->clusters) ctx->depth = std::max(ctx->depth, c.depth);

  ctx->have_tree = true;
  if (info) {
    std::memset(info, 0, sizeof(*info));
    info->n_clusters = int(ctx->clusters.size());
    for (auto& c : ctx->clusters) info->n_leaves += c.son0 < 0;
    info->depth = ctx->depth;
    info->n_blocks = int(ctx->blocks.size());
    info->n_far = int(ctx->far_ids.size());
    info->n_near = int(ctx->near_ids.size());
    for (auto& b : ctx->blocks) {
      const Cluster& A = ctx->clusters[b.row];
      const Cluster& B = ctx->clusters[b.col];
      int64_t m = A.end - A.begin, nn = B.end - B.begin;
      if (b.admissible) info->far_dims += m + nn;
      else info->near_entries += m * nn;
    }
  }
  if (ctx->device < 0) return GCQ_OK;
  ctx->have_tree = false;

  // ---- device panel tables in permuted order
  std::vector<double> cen_p(3 * size_t(n)), h2_p(n), vert_p(9 * size_t(n)), area_p(n),
      q64(28 * size_t(n));
  std::vector<float> c32(3 * size_t(n)), q32(28 * size_t(n)), q4(28 * size_t(n)), n32(3 * size_t(n));
  std::vector<double> n64(3 * size_t(n));
  double rb[7][3], rw[7];
  radon7(rb, rw);
  for (int p = 0; p < n; ++p) {
    int t = ctx->perm[p];
    for (int k = 0; k < 3; ++k) {
      cen_p[k * size_t(n) + p] = cen[3 * t + k];
      c32[k * size_t(n) + p] = float(cen[3 * t + k] - ctx->shift[k]);
    }
    for (int c = 0; c < 9; ++c) vert_p[c * size_t(n) + p] = vert[9 * t + c];
    h2_p[p] = ctx->h2[t];
    area_p[p] = ctx->area[t];
    const double* v = &vert[9 * t];
    {   // unit normal (v1 - v0) x (v2 - v0) / |.|, outward for outward-oriented meshes
      const double ax = v[3] - v[0], ay = v[4] - v[1], az = v[5] - v[2];
      const double bx = v[6] - v[0], by = v[7] - v[1], bz = v[8] - v[2];
      const double cr[3] = {ay * bz - az * by, az * bx - ax * bz, ax * by - ay * bx};
      const double inv = 1.0 / std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
      for (int k = 0; k < 3; ++k) {
        n64[k * size_t(n) + p] = cr[k] * inv;
        n32[k * size_t(n) + p] = float(cr[k] * inv);
      }
    }
    for (int a = 0; a < 7; ++a) {
      for (int k = 0; k < 3; ++k) {
        double x = rb[a][0] * v[k] + rb[a][1] * v[3 + k] + rb[a][2] * v[6 + k];
        q64[(7 * k + a) * size_t(n) + p] = x;
        q32[(7 * k + a) * size_t(n) + p] = float(x - ctx->shift[k]);
        q4[4 * (a * size_t(n) + p) + k] = float(x - ctx->shift[k]);
      }
      double w = rw[a] * ctx->area[t] * INV4PI;
      q64[(21 + a) * size_t(n) + p] = w;
      q32[(21 + a) * size_t(n) + p] = float(w);
      q4[4 * (a * size_t(n) + p) + 3] = float(w);
    }
  }
  std::vector<int32_t> blk(5 * ctx->blocks.size());
  for (size_t b = 0; b < ctx->blocks.size(); ++b) {
    const Cluster& A = ctx->clusters[ctx->blocks[b].row];
    const Cluster& B = ctx->clusters[ctx->blocks[b].col];
    blk[5 * b] = A.begin;
    blk[5 * b + 1] = A.end;
    blk[5 * b + 2] = B.begin;
    blk[5 * b + 3] = B.end;
    blk[5 * b + 4] = (ctx->blocks[b].admissible ? 1 : 0) | (ctx->blocks[b].all_far ? 2 : 0);
  }
  hipStream_t st = ctx->stream;
  GCQ_TRY(upload(ctx->d_cen, cen_p, st));
  GCQ_TRY(upload(ctx->d_h2, h2_p, st));
  GCQ_TRY(upload(ctx->d_vert, vert_p, st));
  GCQ_TRY(upload(ctx->d_area, area_p, st));
  GCQ_TRY(upload(ctx->d_q64, q64, st));
  GCQ_TRY(upload(ctx->d_c32, c32, st));
  GCQ_TRY(upload(ctx->d_q32, q32, st));
  GCQ_TRY(upload(ctx->d_q4, q4, st));
  GCQ_TRY(upload(ctx->d_n64, n64, st));
  GCQ_TRY(upload(ctx->d_n32, n32, st));
  std::vector<int32_t> perm32(ctx->perm.begin(), ctx->perm.end());
  std::vector<int32_t> iperm32(ctx->iperm.begin(), ctx->iperm.end());
  GCQ_TRY(upload(ctx->d_perm, perm32, st));
  GCQ_TRY(upload(ctx->d_iperm, iperm32, st));
  GCQ_TRY(upload(ctx->d_blk, blk, st));
  // near field offsets and the self/near-tier entries of the inadmissible blocks
  {
    ctx->near_off.assign(ctx->near_ids.size(), 0);
    std::vector<SingEntry> sing;
    int64_t acc = 0;
    for (size_t q = 0; q < ctx->near_ids.size(); ++q) {
      const Block& B = ctx->blocks[ctx->near_ids[q]];
      const Cluster& A = ctx->clusters[B.row];
      const Cluster& C = ctx->clusters[B.col];
      const int m = A.end - A.begin, nn = C.end - C.begin;
      ctx->near_off[q] = acc;
      for (int c = 0; c < nn; ++c)
        for (int r = 0; r < m; ++r) {
          const int pi = A.begin + r, pj = C.begin + c;
          const int ti = ctx->perm[pi], tj = ctx->perm[pj];
          double dx = cen[3 * ti] - cen[3 * tj], dy = cen[3 * ti + 1] - cen[3 * tj + 1],
                 dz = cen[3 * ti + 2] - cen[3 * tj + 2];
          double d2 = dx * dx + dy * dy + dz * dz;
          if (pi == pj || d2 < 4.0 * ctx->h2[tj]) sing.push_back(SingEntry{acc + int64_t(c) * m + r, pi, pj});
        }
      acc += int64_t(m) * nn;
    }
    ctx->near_total = acc;
    ctx->n_sing = int64_t(sing.size());
    ctx->sing_off.resize(sing.size());
    for (size_t a = 0; a < sing.size(); ++a) ctx->sing_off[a] = sing[a].off;
    std::vector<int32_t> nid(ctx->near_ids.begin(), ctx->near_ids.end());
    GCQ_TRY(upload(ctx->d_near_off, ctx->near_off, st));
    GCQ_TRY(upload(ctx->d_near_ids, nid, st));
    GCQ_TRY(upload(ctx->d_sing, sing, st));
  }
  GCQ_HIP(hipStreamSynchronize(st));
  ctx->have_tree = true;
  return GCQ_OK;
}

extern "C" {

GCQ_API const char* gcq_last_error(void) { return gcq::g_err.c_str(); }

GCQ_API int gcq_create(int device, void* hip_stream, gcq_context** out) {
  if (!out) return fail(GCQ_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (device == -1) {  // host-only context: geometry, trees and features, no device work
    gcq_context* ctx = new (std::nothrow) gcq_context();
    if (!ctx) return fail(GCQ_ERR_NOMEM, "host allocation failed");
    ctx->device = -1;
    *out = ctx;
    return GCQ_OK;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
    (void)hipGetLastError();
    return fail(GCQ_ERR_HIP, "no HIP device available");
  }
  if (device < 0 || device >= ndev) return fail(GCQ_ERR_ARG, "device %d out of range", device);
  GCQ_HIP(hipSetDevice(device));
  gcq_context* ctx = new (std::nothrow) gcq_context();
  if (!ctx) return fail(GCQ_ERR_NOMEM, "host allocation failed");
  ctx->device = device;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) ctx->cus = prop.multiProcessorCount;
  }
  if (hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess ||
      hipEventCreate(&ctx->evm) != hipSuccess) {
    delete ctx;
    return fail(GCQ_ERR_HIP, "hipEventCreate failed");
  }
  Consts K;
  build_consts(K);
  int st = noalloc_scratch_init(device);
  if (st == GCQ_OK) st = ctx->d_consts.ensure(sizeof(Consts));
  if (st == GCQ_OK &&
      hipMemcpy(ctx->d_consts.p, &K, sizeof(Consts), hipMemcpyHostToDevice) != hipSuccess)
    st = fail(GCQ_ERR_HIP, "upload of constant tables failed");
  if (st != GCQ_OK) {
    gcq_destroy(ctx);
    return st;
  }
  *out = ctx;
  return GCQ_OK;
}

GCQ_API int gcq_destroy(gcq_context* ctx) {
  if (!ctx) return GCQ_OK;
  if (ctx->device < 0) {
    delete ctx;
    return GCQ_OK;
  }
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  else (void)hipDeviceSynchronize();
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  if (ctx->evm) (void)hipEventDestroy(ctx->evm);
  if (ctx->evfork) (void)hipEventDestroy(ctx->evfork);
  for (int i = 0; i < 3; ++i) {
    if (ctx->side[i]) {
      (void)hipStreamSynchronize(ctx->side[i]);
      (void)hipStreamDestroy(ctx->side[i]);
    }
    if (ctx->evjoin[i]) (void)hipEventDestroy(ctx->evjoin[i]);
  }
  delete ctx;  // DevBuf destructors free device memory
  return GCQ_OK;
}

GCQ_API int gcq_set_tuning(gcq_context* ctx, const gcq_tuning* tuning) {
  if (!ctx || !tuning) return fail(GCQ_ERR_ARG, "ctx or tuning is NULL");
  for (int c = 0; c < 4; ++c) {
    const int w = tuning->aca3d_waves[c];
    if (w != 1 && w != 2 && w != 4 && w != 8)
      return fail(GCQ_ERR_ARG, "aca3d_waves[%d] = %d is not 1, 2, 4 or 8", c, w);
  }
  if (tuning->aca3d_stack_slices < 1 || tuning->aca3d_stack_slices > 64)
    return fail(GCQ_ERR_ARG, "aca3d_stack_slices = %d is not in 1..64", tuning->aca3d_stack_slices);
  if (tuning->aca_waves != 1 && tuning->aca_waves != 2 && tuning->aca_waves != 4)
    return fail(GCQ_ERR_ARG, "aca_waves = %d is not 1, 2 or 4", tuning->aca_waves);
  if (tuning->product_graph != 0 && tuning->product_graph != 1)
    return fail(GCQ_ERR_ARG, "product_graph = %d is not 0 or 1", tuning->product_graph);
  if (tuning->product_cols_per_wave != 32 && tuning->product_cols_per_wave != 64)
    return fail(GCQ_ERR_ARG, "product_cols_per_wave = %d is not 32 or 64", tuning->product_cols_per_wave);
  if (tuning->product_cols_per_wave != ctx->tune.product_cols_per_wave) ctx->F.graphs.clear();
  ctx->tune = *tuning;
  return GCQ_OK;
}

GCQ_API int gcq_get_tuning(gcq_context* ctx, gcq_tuning* tuning) {
  if (!ctx || !tuning) return fail(GCQ_ERR_ARG, "ctx or tuning is NULL");
  *tuning = ctx->tune;
  return GCQ_OK;
}

GCQ_API double gcq_kernel_ms(gcq_context* ctx, const char* name) {
  if (!ctx || !name) return -1.0;
  auto it = ctx->kernel_ms.find(name);
  return it == ctx->kernel_ms.end() ? -1.0 : it->second;
}

GCQ_API int gcq_upload_mesh(gcq_context* ctx, const double* xyz, int64_t n_vertices,
                            const int32_t* tri, int64_t n_triangles, double wave_speed) {
#pragma clang fp contract(off)
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!xyz || !tri) return fail(GCQ_ERR_ARG, "xyz/tri is NULL");
  if (n_vertices < 3 || n_triangles < 1 || n_triangles > (int64_t(1) << 30))
    return fail(GCQ_ERR_ARG, "bad mesh sizes (%lld vertices, %lld triangles)",
                (long long)n_vertices, (long long)n_triangles);
  if (!(wave_speed > 0.0) || !std::isfinite(wave_speed))
    return fail(GCQ_ERR_ARG, "wave speed must be positive and finite");
  // invalidate everything downstream
  ctx->have_mesh = ctx->have_tree = false;
  ctx->H.valid = ctx->F.valid = false;
  ctx->F.drop_product_state();
  const int n = int(n_triangles);
  for (int64_t i = 0; i < 3 * n_vertices; ++i)
    if (!std::isfinite(xyz[i])) return fail(GCQ_ERR_NUMERIC, "non-finite vertex coordinate");
  for (int64_t i = 0; i < 3 * n_triangles; ++i)
    if (tri[i] < 0 || tri[i] >= n_vertices)
      return fail(GCQ_ERR_ARG, "triangle vertex id %d out of range", tri[i]);
  ctx->n = n;
  ctx->nv = n_vertices;
  ctx->c = wave_speed;
  ctx->cen.assign(3 * size_t(n), 0.0);
  ctx->h2.assign(n, 0.0);
  ctx->area.assign(n, 0.0);
  ctx->vert.assign(9 * size_t(n), 0.0);
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  for (int64_t v = 0; v < n_vertices; ++v)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], xyz[3 * v + k]);
      hi[k] = std::max(hi[k], xyz[3 * v + k]);
    }
  for (int k = 0; k < 3; ++k) ctx->shift[k] = 0.5 * (lo[k] + hi[k]);
  for (int t = 0; t < n; ++t) {
    const double* a = xyz + 3 * int64_t(tri[3 * t]);
    const double* b = xyz + 3 * int64_t(tri[3 * t + 1]);
    const double* c = xyz + 3 * int64_t(tri[3 * t + 2]);
    for (int k = 0; k < 3; ++k) {
      ctx->cen[3 * t + k] = (a[k] + b[k] + c[k]) / 3.0;
      ctx->vert[9 * t + k] = a[k];
      ctx->vert[9 * t + 3 + k] = b[k];
      ctx->vert[9 * t + 6 + k] = c[k];
    }
    double e0 = (b[0] - a[0]) * (b[0] - a[0]) + (b[1] - a[1]) * (b[1] - a[1]) +
                (b[2] - a[2]) * (b[2] - a[2]);
    double e1 = (c[0] - b[0]) * (c[0] - b[0]) + (c[1] - b[1]) * (c[1] - b[1]) +
                (c[2] - b[2]) * (c[2] - b[2]);
    double e2 = (a[0] - c[0]) * (a[0] - c[0]) + (a[1] - c[1]) * (a[1] - c[1]) +
                (a[2] - c[2]) * (a[2] - c[2]);
    ctx->h2[t] = std::max(std::max(e0, e1), e2);
    double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
    double vx = c[0] - a[0], vy = c[1] - a[1], vz = c[2] - a[2];
    double cx = uy * vz - uz * vy, cy = uz * vx - ux * vz, cz = ux * vy - uy * vx;
    ctx->area[t] = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
    if (!(ctx->area[t] > 0.0)) return fail(GCQ_ERR_NUMERIC, "triangle %d has zero area", t);
  }
  ctx->have_mesh = true;
  ctx->have_tree = false;
  return GCQ_OK;
}

GCQ_API int gcq_set_frequencies(gcq_context* ctx, const gcq_c128* s, int32_t n_freq,
                                int32_t use_conjugate_symmetry) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!s || n_freq < 1) return fail(GCQ_ERR_ARG, "need at least one frequency");
  for (int k = 0; k < n_freq; ++k) {
    if (!std::isfinite(s[k].re) || !std::isfinite(s[k].im))
      return fail(GCQ_ERR_ARG, "frequency %d is not finite", k);
    if (!(s[k].re > 0.0)) return fail(GCQ_ERR_ARG, "frequency %d has Re s <= 0", k);
  }
  ctx->H.valid = ctx->F.valid = false;
  ctx->F.drop_product_state();
  ctx->L = n_freq;
  ctx->s.resize(n_freq);
  for (int k = 0; k < n_freq; ++k) ctx->s[k] = {s[k].re, s[k].im};
  ctx->rep.resize(n_freq);
  ctx->conj.assign(n_freq, 0);
  for (int k = 0; k < n_freq; ++k) ctx->rep[k] = k;
  if (use_conjugate_symmetry) {
    for (int k = n_freq / 2 + 1; k < n_freq; ++k) {
      int j = n_freq - k;
      std::complex<double> d = ctx->s[k] - std::conj(ctx->s[j]);
      if (std::abs(d) <= 1e-12 * std::abs(ctx->s[j])) {
        ctx->rep[k] = j;
        ctx->conj[k] = 1;
      }
    }
  }
  ctx->K.clear();
  for (int k = 0; k < n_freq; ++k)
    if (ctx->rep[k] == k) ctx->K.push_back(k);
  std::vector<int> pos(n_freq, -1);
  for (size_t p = 0; p < ctx->K.size(); ++p) pos[ctx->K[p]] = int(p);
  ctx->kpos.resize(n_freq);
  for (int k = 0; k < n_freq; ++k) ctx->kpos[k] = pos[ctx->rep[k]];
  ctx->have_freq = true;
  return GCQ_OK;
}

GCQ_API int gcq_build_cluster_tree(gcq_context* ctx, int32_t leaf_size, double eta,
                                   gcq_tree_info* info) {
#pragma clang fp contract(off)
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!ctx->have_mesh) return fail(GCQ_ERR_STATE, "upload a mesh first");
  if (leaf_size < 1) return fail(GCQ_ERR_ARG, "leaf_size must be >= 1");
  if (!(eta > 0.0) || !std::isfinite(eta)) return fail(GCQ_ERR_ARG, "eta must be positive");
  if (ctx->device >= 0) GCQ_HIP(hipSetDevice(ctx->device));
  ctx->have_tree = false;
  ctx->H.valid = ctx->F.valid = false;
  ctx->F.drop_product_state();
  const int n = ctx->n;
  ctx->leaf = leaf_size;
  ctx->eta = eta;
  ctx->perm.resize(n);
  std::iota(ctx->perm.begin(), ctx->perm.end(), 0);
  ctx->clusters.clear();
  std::vector<double> maxh2;
  const std::vector<double>& cen = ctx->cen;
  const std::vector<double>& vert = ctx->vert;

  // cluster tree: recursive bisection along the longest centroid extent
  std::vector<std::pair<double, int>> keys;
  std::function<int(int, int, int)> build = [&](int lo, int hi, int depth) -> int {
    int id = int(ctx->clusters.size());
    ctx->clusters.push_back(Cluster{lo, hi, -1, -1, depth, {1e300, 1e300, 1e300},
                                    {-1e300, -1e300, -1e300}});
    maxh2.push_back(0.0);
    double cl[3] = {1e300, 1e300, 1e300}, ch[3] = {-1e300, -1e300, -1e300};
    double mh = 0.0;
    Cluster c = ctx->clusters[id];
    for (int p = lo; p < hi; ++p) {
      int t = ctx->perm[p];
      for (int k = 0; k < 3; ++k) {
        cl[k] = std::min(cl[k], cen[3 * t + k]);
        ch[k] = std::max(ch[k], cen[3 * t + k]);
        for (int v = 0; v < 3; ++v) {
          c.bmin[k] = std::min(c.bmin[k], vert[9 * t + 3 * v + k]);
          c.bmax[k] = std::max(c.bmax[k], vert[9 * t + 3 * v + k]);
        }
      }
      mh = std::max(mh, ctx->h2[t]);
    }
    ctx->clusters[id] = c;
    maxh2[id] = mh;
    const int cnt = hi - lo;
    if (cnt <= leaf_size) return id;
    int axis = 0;
    double best = ch[0] - cl[0];
    for (int k = 1; k < 3; ++k)
      if (ch[k] - cl[k] > best) {
        best = ch[k] - cl[k];
        axis = k;
      }
    keys.resize(cnt);
    for (int p = lo; p < hi; ++p) keys[p - lo] = {cen[3 * ctx->perm[p] + axis], ctx->perm[p]};
    std::sort(keys.begin(), keys.end());
    for (int p = lo; p < hi; ++p) ctx->perm[p] = keys[p - lo].second;
    const int mid = lo + cnt / 2;
    int s0 = build(lo, mid, depth + 1);
    int s1 = build(mid, hi, depth + 1);
    ctx->clusters[id].son0 = s0;
    ctx->clusters[id].son1 = s1;
    return id;
  };
  build(0, n, 0);

  // block cluster tree: admissibility on squared box diagonal / distance
  const double eta2 = eta * eta;
  auto diam2 = [&](const Cluster& c) {
    double dx = c.bmax[0] - c.bmin[0], dy = c.bmax[1] - c.bmin[1], dz = c.bmax[2] - c.bmin[2];
    return dx * dx + dy * dy + dz * dz;
  };
  auto dist2 = [&](const Cluster& a, const Cluster& b) {
    double g[3];
    for (int k = 0; k < 3; ++k)
      g[k] = std::max(0.0, std::max(a.bmin[k] - b.bmax[k], b.bmin[k] - a.bmax[k]));
    return g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  };
  ctx->blocks.clear();
  std::function<void(int, int)> rec = [&](int a, int b) {
    const Cluster& A = ctx->clusters[a];
    const Cluster& B = ctx->clusters[b];
    double d2 = dist2(A, B);
    bool adm = d2 > 0.0 && std::min(diam2(A), diam2(B)) <= eta2 * d2;
    bool leafpair = A.son0 < 0 || B.son0 < 0;
    if (adm || leafpair) {
      Block blk;
      blk.row = a;
      blk.col = b;
      blk.admissible = adm;
      blk.all_far = d2 > 0.0 && d2 >= 4.0 * maxh2[b] * (1.0 + 1e-12);
      ctx->blocks.push_back(blk);
      return;
    }
    rec(A.son0, B.son0);
    rec(A.son0, B.son1);
    rec(A.son1, B.son0);
    rec(A.son1, B.son1);
  };
  rec(0, 0);

  return finish_tree(ctx, info);
}

GCQ_API int gcq_upload_cluster_tree(gcq_context* ctx, const int32_t* perm, int32_t n_clusters,
                                    const int32_t* cl_begin, const int32_t* cl_end,
                                    const int32_t* cl_son, int32_t n_blocks, const int32_t* blk_row,
                                    const int32_t* blk_col, const uint8_t* blk_admissible,
                                    gcq_tree_info* info) {
#pragma clang fp contract(off)
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!ctx->have_mesh) return fail(GCQ_ERR_STATE, "upload a mesh first");
  if (!perm || !cl_begin || !cl_end || !cl_son || !blk_row || !blk_col || !blk_admissible)
    return fail(GCQ_ERR_ARG, "NULL tree array");
  if (n_clusters < 1 || n_blocks < 1) return fail(GCQ_ERR_ARG, "need at least one cluster and one block");
  const int n = ctx->n;
  // perm: a permutation of 0..n-1
  {
    std::vector<char> seen(n, 0);
    for (int p = 0; p < n; ++p) {
      if (perm[p] < 0 || perm[p] >= n || seen[perm[p]])
        return fail(GCQ_ERR_ARG, "perm is not a permutation of 0..%d", n - 1);
      seen[perm[p]] = 1;
    }
  }
  // clusters: root 0 = [0, n); sons split their parent's range in two, carry
  // larger indices than the parent, and every cluster but the root has one parent
  if (cl_begin[0] != 0 || cl_end[0] != n) return fail(GCQ_ERR_ARG, "cluster 0 must be the root [0, n)");
  std::vector<int> parents(n_clusters, 0), depth(n_clusters, 0);
  for (int c = 0; c < n_clusters; ++c) {
    if (!(0 <= cl_begin[c] && cl_begin[c] < cl_end[c] && cl_end[c] <= n))
      return fail(GCQ_ERR_ARG, "cluster %d has an empty or out-of-range index range", c);
    const int s0 = cl_son[2 * c], s1 = cl_son[2 * c + 1];
    if (s0 < 0 && s1 < 0) continue;
    if (s0 <= c || s1 <= c || s0 >= n_clusters || s1 >= n_clusters || s0 == s1)
      return fail(GCQ_ERR_ARG, "cluster %d: sons must be two distinct clusters of larger index", c);
    if (cl_begin[s0] != cl_begin[c] || cl_end[s0] != cl_begin[s1] || cl_end[s1] != cl_end[c])
      return fail(GCQ_ERR_ARG, "cluster %d: its sons do not split its range in two", c);
    ++parents[s0];
    ++parents[s1];
    depth[s0] = depth[s1] = depth[c] + 1;   // parents precede their sons
  }
  for (int c = 1; c < n_clusters; ++c)
    if (parents[c] != 1) return fail(GCQ_ERR_ARG, "cluster %d has %d parents", c, parents[c]);
  // boxes of all vertices and the largest squared longest edge, per cluster
  std::vector<Cluster> cl(n_clusters);
  std::vector<double> maxh2(n_clusters, 0.0);
  for (int c = 0; c < n_clusters; ++c) {
    Cluster& C = cl[c];
    C = Cluster{cl_begin[c], cl_end[c], cl_son[2 * c], cl_son[2 * c + 1], depth[c],
                {1e300, 1e300, 1e300}, {-1e300, -1e300, -1e300}};
    for (int p = C.begin; p < C.end; ++p) {
      const int t = perm[p];
      for (int k = 0; k < 3; ++k)
        for (int v = 0; v < 3; ++v) {
          C.bmin[k] = std::min(C.bmin[k], ctx->vert[9 * t + 3 * v + k]);
          C.bmax[k] = std::max(C.bmax[k], ctx->vert[9 * t + 3 * v + k]);
        }
      maxh2[c] = std::max(maxh2[c], ctx->h2[t]);
    }
  }
  auto dist2 = [&](const Cluster& a, const Cluster& b) {
    double g[3];
    for (int k = 0; k < 3; ++k)
      g[k] = std::max(0.0, std::max(a.bmin[k] - b.bmax[k], b.bmin[k] - a.bmax[k]));
    return g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  };
  // blocks: cluster pairs; an admissible one needs boxes at positive distance
  std::vector<Block> blocks(n_blocks);
  std::unordered_map<int64_t, int> where;
  for (int b = 0; b < n_blocks; ++b) {
    const int r = blk_row[b], c = blk_col[b];
    if (r < 0 || r >= n_clusters || c < 0 || c >= n_clusters)
      return fail(GCQ_ERR_ARG, "block %d names a cluster out of range", b);
    if (blk_admissible[b] > 1) return fail(GCQ_ERR_ARG, "block %d: admissible must be 0 or 1", b);
    const double d2 = dist2(cl[r], cl[c]);
    if (blk_admissible[b] && !(d2 > 0.0))
      return fail(GCQ_ERR_ARG, "block %d is marked admissible but its clusters' boxes touch", b);
    if (!where.emplace(int64_t(r) * n_clusters + c, b).second)
      return fail(GCQ_ERR_ARG, "block %d repeats a cluster pair", b);
    blocks[b].row = r;
    blocks[b].col = c;
    blocks[b].admissible = blk_admissible[b] != 0;
    blocks[b].all_far = d2 > 0.0 && d2 >= 4.0 * maxh2[c] * (1.0 + 1e-12);
  }
  // the blocks are the leaves of a block tree over the cluster tree: from
  // (root, root), a pair that is not a block is split through the sons of
  // whichever clusters have them; every pair reached must be a block or
  // splittable, and every block must be reached, so they tile [0, n)^2 once
  {
    std::vector<char> used(n_blocks, 0);
    std::vector<std::pair<int, int>> stack{{0, 0}};
    int reached = 0;
    while (!stack.empty()) {
      const auto [a, c] = stack.back();
      stack.pop_back();
      const auto it = where.find(int64_t(a) * n_clusters + c);
      if (it != where.end()) {
        used[it->second] = 1;
        ++reached;
        continue;
      }
      const bool sa = cl[a].son0 >= 0, sc = cl[c].son0 >= 0;
      if (!sa && !sc)
        return fail(GCQ_ERR_ARG, "the blocks do not cover the pair of leaf clusters (%d, %d)", a, c);
      const int as[2] = {sa ? cl[a].son0 : a, sa ? cl[a].son1 : a};
      const int cs[2] = {sc ? cl[c].son0 : c, sc ? cl[c].son1 : c};
      for (int x = (sa ? 1 : 0); x >= 0; --x)
        for (int y = (sc ? 1 : 0); y >= 0; --y) stack.push_back({as[x], cs[y]});
    }
    if (reached != n_blocks)
      return fail(GCQ_ERR_ARG, "%d blocks lie inside other blocks (the blocks overlap)", n_blocks - reached);
  }
  if (ctx->device >= 0) GCQ_HIP(hipSetDevice(ctx->device));
  ctx->have_tree = false;
  ctx->H.valid = ctx->F.valid = false;
  ctx->F.drop_product_state();
  ctx->perm.assign(perm, perm + n);
  ctx->clusters = std::move(cl);
  ctx->blocks = std::move(blocks);
  ctx->leaf = 0;
  for (auto& C : ctx->clusters)
    if (C.son0 < 0) ctx->leaf = std::max(ctx->leaf, C.end - C.begin);
  ctx->eta = 0.0;
  return finish_tree(ctx, info);
}

GCQ_API int gcq_trim(gcq_context* ctx, int32_t release_faces) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  GCQ_HIP(hipSetDevice(ctx->device));
  GCQ_HIP(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < 3; ++i)
    if (ctx->side[i]) GCQ_HIP(hipStreamSynchronize(ctx->side[i]));
  ctx->scratchA.release();
  ctx->scratchB.release();
  ctx->scratchC.release();
  ctx->scratchD.release();
  ctx->scratchT.release();
  ctx->F.graphs.clear();       // they refer to the product buffers released below
  ctx->F.meta_valid = false;
  ctx->F.bf_valid = false;
  ctx->F.bfpool.release();
  ctx->F.bftbuf.release();
  ctx->F.pxy.release();
  ctx->Mf.release_work();
  if (release_faces) {
    HFaces& H = ctx->H;
    H.valid = false;
    H.factors.release();
    H.near.release();
    H.d_off.release();
    H.d_rank.release();
    H.d_near_off.release();
    H.d_sig.release();
  }
  return GCQ_OK;
}

GCQ_API int gcq_get_tree(gcq_context* ctx, int32_t* perm, int32_t* blocks) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  if (!ctx->have_tree) return fail(GCQ_ERR_STATE, "build the cluster tree first");
  if (perm)
    for (int p = 0; p < ctx->n; ++p) perm[p] = ctx->perm[p];
  if (blocks)
    for (size_t b = 0; b < ctx->blocks.size(); ++b) {
      const Cluster& A = ctx->clusters[ctx->blocks[b].row];
      const Cluster& B = ctx->clusters[ctx->blocks[b].col];
      blocks[5 * b] = A.begin;
      blocks[5 * b + 1] = A.end;
      blocks[5 * b + 2] = B.begin;
      blocks[5 * b + 3] = B.end;
      blocks[5 * b + 4] = ctx->blocks[b].admissible ? 1 : 0;
    }
  return GCQ_OK;
}

}  // extern "C"
