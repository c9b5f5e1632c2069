// Dense entries V(s_f)[rows[a], cols[b]] (single layer) and K(s_f)[rows[a],
// cols[b]] (double layer) for index and frequency lists.
#include <mutex>

#include "internal.h"

namespace gcq {

// Staging memory of gcq_assemble_slices_noalloc: the permuted index lists and
// the frequencies of a call live here instead of in buffers the library
// allocates.  Each GPU holds its own copy of the array for the life of the
// process; host code reaches it only through the address hipGetSymbolAddress
// returns for that device (the array's name is not a device address there).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// once per device, with that device current (called by gcq_create)
int noalloc_scratch_init(int device) {
  if (device < 0 || device >= NOALLOC_MAX_DEVICES) return fail(GCQ_ERR_UNSUPPORTED, "device %d beyond %d", device,
                                                               NOALLOC_MAX_DEVICES);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return GCQ_OK;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return fail(GCQ_ERR_HIP, "hipGetSymbolAddress of the staging array failed: %s", hipGetErrorString(e));
  }
  g_scratch_ptr[device] = p;
  return GCQ_OK;
}

static void* scratch_ptr(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return (device >= 0 && device < NOALLOC_MAX_DEVICES) ? g_scratch_ptr[device] : nullptr;
}

// one thread per (a, b); the frequencies loop inside so that the geometry of
// the pair is loaded once.  out[(f * ncol + b) * nrow + a].
template <typename T, bool DLP>
__global__ void __launch_bounds__(256) assemble_kernel(Tab tab, const int* __restrict__ prow,
                                                       const int* __restrict__ pcol, int64_t nrow,
                                                       int64_t ncol, const double2* __restrict__ sig,
                                                       int nf, cpx<T>* __restrict__ out) {
  const int64_t id = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= nrow * ncol) return;
  const int64_t a = id % nrow, b = id / nrow;
  const int pi = prow[a], pj = pcol[b];
  for (int f = 0; f < nf; ++f) {
    double2 s = sig[f];
    out[(int64_t(f) * ncol + b) * nrow + a] =
        DLP ? dlp_entry_part<T>(tab, pi, pj, s.x, s.y, false, 0, 1) : entry<T>(tab, pi, pj, s.x, s.y, false);
  }
}

// staged: the index lists and frequencies go to the per-device staging array
// (no allocation, no synchronisation) instead of the context's buffers
template <bool DLP>
static int assemble(gcq_context* ctx, const int32_t* rows, int64_t n_rows, const int32_t* cols, int64_t n_cols,
                    const int32_t* freq_idx, int32_t n_fidx, int32_t precision, void* out_dev,
                    bool staged = false) {
  if (!ctx) return fail(GCQ_ERR_ARG, "ctx is NULL");
  GCQ_NEED_DEVICE(ctx);
  if (!ctx->have_tree) return fail(GCQ_ERR_STATE, "build the cluster tree first");
  if (!ctx->have_freq) return fail(GCQ_ERR_STATE, "set the frequencies first");
  if (precision != GCQ_C128 && precision != GCQ_C64)
    return fail(GCQ_ERR_ARG, "unknown precision %d", precision);
  if (n_rows < 0 || n_cols < 0 || n_fidx < 0) return fail(GCQ_ERR_ARG, "negative size");
  if (n_rows == 0 || n_cols == 0 || n_fidx == 0) return GCQ_OK;
  if (!rows || !cols || !freq_idx) return fail(GCQ_ERR_ARG, "index list is NULL");
  GCQ_HIP(hipSetDevice(ctx->device));
  GCQ_TRY(check_device_ptr(ctx, out_dev, "out_dev"));
  std::vector<int32_t> pr(n_rows), pc(n_cols);
  for (int64_t a = 0; a < n_rows; ++a) {
    if (rows[a] < 0 || rows[a] >= ctx->n) return fail(GCQ_ERR_ARG, "row index out of range");
    pr[a] = ctx->iperm[rows[a]];
  }
  for (int64_t b = 0; b < n_cols; ++b) {
    if (cols[b] < 0 || cols[b] >= ctx->n) return fail(GCQ_ERR_ARG, "column index out of range");
    pc[b] = ctx->iperm[cols[b]];
  }
  std::vector<double2> sig(n_fidx);
  for (int f = 0; f < n_fidx; ++f) {
    if (freq_idx[f] < 0 || freq_idx[f] >= ctx->L)
      return fail(GCQ_ERR_ARG, "frequency index out of range");
    std::complex<double> sg = ctx->s[freq_idx[f]] / ctx->c;
    sig[f] = make_double2(sg.real(), sg.imag());
  }
  const int64_t total = n_rows * n_cols;
  const int64_t nblk = (total + 255) / 256;
  if (nblk > 0x7fffffff) return fail(GCQ_ERR_ARG, "request too large");
  const int* d_rows;
  const int* d_cols;
  const double2* d_sig;
  if (staged) {
    // [rows | cols | frequencies], each part on a 256-byte boundary
    const size_t o1 = (size_t(n_rows) * 4 + 255) / 256 * 256;
    const size_t o2 = o1 + (size_t(n_cols) * 4 + 255) / 256 * 256;
    const size_t need = o2 + size_t(n_fidx) * sizeof(double2);
    if (need > NOALLOC_SCRATCH_BYTES)
      return fail(GCQ_ERR_ARG, "request needs %zu bytes of staging, the limit is %zu", need,
                  NOALLOC_SCRATCH_BYTES);
    unsigned char* base = static_cast<unsigned char*>(scratch_ptr(ctx->device));
    if (!base) return fail(GCQ_ERR_STATE, "the staging array of device %d is not set up", ctx->device);
    GCQ_HIP(hipMemcpyAsync(base, pr.data(), sizeof(int32_t) * n_rows, hipMemcpyHostToDevice, ctx->stream));
    GCQ_HIP(hipMemcpyAsync(base + o1, pc.data(), sizeof(int32_t) * n_cols, hipMemcpyHostToDevice, ctx->stream));
    GCQ_HIP(hipMemcpyAsync(base + o2, sig.data(), sizeof(double2) * n_fidx, hipMemcpyHostToDevice, ctx->stream));
    d_rows = reinterpret_cast<const int*>(base);
    d_cols = reinterpret_cast<const int*>(base + o1);
    d_sig = reinterpret_cast<const double2*>(base + o2);
  } else {
    GCQ_TRY(upload(ctx->scratchA, pr, ctx->stream));
    GCQ_TRY(upload(ctx->scratchB, pc, ctx->stream));
    GCQ_TRY(upload(ctx->scratchC, sig, ctx->stream));
    d_rows = ctx->scratchA.as<int>();
    d_cols = ctx->scratchB.as<int>();
    d_sig = ctx->scratchC.as<double2>();
    GCQ_TRY(timed_begin(ctx));
  }
  if (precision == GCQ_C128)
    hipLaunchKernelGGL((assemble_kernel<double, DLP>), dim3(unsigned(nblk)), dim3(256), 0, ctx->stream,
                       ctx->tab(), d_rows, d_cols, n_rows, n_cols, d_sig, n_fidx,
                       reinterpret_cast<cpx<double>*>(out_dev));
  else
    hipLaunchKernelGGL((assemble_kernel<float, DLP>), dim3(unsigned(nblk)), dim3(256), 0, ctx->stream,
                       ctx->tab(), d_rows, d_cols, n_rows, n_cols, d_sig, n_fidx,
                       reinterpret_cast<cpx<float>*>(out_dev));
  GCQ_HIP(hipGetLastError());
  if (!staged) timed_end(ctx, DLP ? "assemble_dlp" : "assemble");
  return GCQ_OK;
}

}  // namespace gcq

using namespace gcq;

extern "C" GCQ_API int gcq_assemble_slices(gcq_context* ctx, const int32_t* rows, int64_t n_rows,
                                           const int32_t* cols, int64_t n_cols,
                                           const int32_t* freq_idx, int32_t n_fidx,
                                           int32_t precision, void* out_dev) {
  return assemble<false>(ctx, rows, n_rows, cols, n_cols, freq_idx, n_fidx, precision, out_dev);
}

extern "C" GCQ_API int gcq_assemble_dlp_slices(gcq_context* ctx, const int32_t* rows, int64_t n_rows,
                                               const int32_t* cols, int64_t n_cols,
                                               const int32_t* freq_idx, int32_t n_fidx,
                                               int32_t precision, void* out_dev) {
  return assemble<true>(ctx, rows, n_rows, cols, n_cols, freq_idx, n_fidx, precision, out_dev);
}

extern "C" GCQ_API int gcq_assemble_slices_noalloc(gcq_context* ctx, const int32_t* rows, int64_t n_rows,
                                                   const int32_t* cols, int64_t n_cols,
                                                   const int32_t* freq_idx, int32_t n_fidx,
                                                   int32_t precision, void* out_dev) {
  return assemble<false>(ctx, rows, n_rows, cols, n_cols, freq_idx, n_fidx, precision, out_dev, true);
}
