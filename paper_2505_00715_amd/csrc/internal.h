// Host-side state of a gcqbem context and helpers shared by the API files.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/gcqbem.h"
#include "device_common.h"

namespace gcq {

// ---- errors -------------------------------------------------------------------
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

#define GCQ_HIP(call)                                                            \
  do {                                                                           \
    hipError_t e_ = (call);                                                      \
    if (e_ != hipSuccess)                                                        \
      return ::gcq::fail(GCQ_ERR_HIP, "%s failed: %s (%s:%d)", #call,            \
                         hipGetErrorString(e_), __FILE__, __LINE__);             \
  } while (0)

#define GCQ_TRY(call)          \
  do {                         \
    int s_ = (call);           \
    if (s_ < 0) return s_;     \
  } while (0)

// ---- device memory owned by the library ----------------------------------------
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // (re)allocate to at least `n` bytes; contents are not preserved
  int ensure(size_t n) {
    if (n <= bytes && p) return GCQ_OK;
    release();
    if (n == 0) n = 256;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(GCQ_ERR_NOMEM, "hipMalloc of %zu bytes failed: %s", n, hipGetErrorString(e));
    }
    bytes = n;
    return GCQ_OK;
  }
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

template <typename T>
int upload(DevBuf& b, const std::vector<T>& v, hipStream_t st) {
  GCQ_TRY(b.ensure(v.size() * sizeof(T)));
  if (!v.empty())
    GCQ_HIP(hipMemcpyAsync(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
  return GCQ_OK;
}

// ---- tree ------------------------------------------------------------------------
struct Cluster {
  int begin, end, son0, son1, depth;
  double bmin[3], bmax[3];
};
struct Block {
  int row, col;      // cluster ids
  bool admissible;
  bool all_far;      // no self or near-tier pair inside (guaranteed by box distance)
};

// ---- 3D-ACA work descriptors (shared by the ACA-based and the FMM-based variants) ----
constexpr int R3_MAX = 64;      // terms per block the kernel can hold
constexpr int NK_MAX = 2048;    // frequencies in K

struct BlockDesc3 {
  int rb, m, cb, n;
  int admissible, all_far;
  int sres;        // admissible: columns reserved for the block's stacked slice factors
  int pad;
};

// A term of a block.  Far blocks keep their slices' factors stacked: the
// block reserves U columns (m x sres) and V columns (n x sres) in the pool,
// and slice d owns columns [c_d, c_d + rank_d) of both.
struct Term3 {
  int64_t slice;   // pool offset (elements) of the slice: dense m x n, or its first Ubar column
  int64_t vslice;  // far: pool offset of its first Vbar column
  int64_t fiber;   // pool offset of the fiber (nK elements)
  int rank;        // slice rank (far) or -1 (dense)
  int freq;        // position in K of the frequency the slice was taken at
};

// ---- per-frequency H-matrices (aca_blocks) ---------------------------------------------
struct HFaces {
  bool valid = false;
  bool dlp = false;              // faces of the double layer (GCQ_FLAG_DOUBLE_LAYER)
  int precision = GCQ_C128;
  std::vector<int> freqs;        // representative frequencies held (positions in K order)
  std::vector<int> fslot;        // L -> slot in freqs or -1
  // far: per (far block f, slot q): offset (in complex elements) and rank
  std::vector<int64_t> off;      // n_far * nslot
  std::vector<int> rank;         // n_far * nslot
  DevBuf d_off, d_rank;
  DevBuf factors;                // pool: U (m x r) then V (n x r), column-major, per pair
  // near: dense blocks per slot, column-major |I| x |J|
  std::vector<int64_t> near_off; // n_near (offset within one slot)
  int64_t near_slot_elems = 0;
  DevBuf d_near_off;
  DevBuf near;                   // nslot * near_slot_elems
  DevBuf d_sig;                  // sigma = s / c of each slot (near-field kernels)
  int64_t storage_bytes = 0;
};

// ---- 3D-ACA result --------------------------------------------------------------------
// instantiated graphs of the per-frequency product, keyed by the caller's
// buffers and the precision; destroyed with the operator they were captured on
struct ProductGraphs {
  struct Entry {
    const void* X;
    void* Y;
    int precision;
    hipGraphExec_t exec;
  };
  std::vector<Entry> e;
  hipStream_t cap = nullptr;   // capture stream
  ~ProductGraphs() {
    clear();
    if (cap) (void)hipStreamDestroy(cap);
  }
  void clear() {
    for (auto& x : e) (void)hipGraphExecDestroy(x.exec);
    e.clear();
  }
};

struct Faces3D {
  bool dlp = false;              // built for the double layer (GCQ_FLAG_DOUBLE_LAYER)
  bool valid = false;
  int precision = GCQ_C128;
  int nK = 0;
  // per block: rank r_b, first term index into the term arrays
  std::vector<int> brank, bterm;
  // per term: frequency position, slice rank (far) or -1 (near), offset of the
  // slice data (complex elements), offset of the fiber (complex elements)
  std::vector<int> tfreq, trank;
  std::vector<int64_t> toff, tvoff, tfoff;   // slice (dense or Ubar), Vbar, fiber offsets
  DevBuf d_brank, d_bterm, d_trank, d_toff, d_tvoff, d_tfoff;
  DevBuf slices;                 // far: U (m x r) then V (n x r); near: dense m x n
  DevBuf fibers;                 // per term: nK complex
  // product tables: per far block its stacked columns (U column offset, V
  // column offset, fiber offset), blocks ordered by work, largest first
  DevBuf d_cols, d_bcol, d_mvorder;
  // the product's own buffers: frequency-major copies of X and Y, frequency
  // tables (position in K, conjugation flag); fixed while the operator lives
  DevBuf pxy, pmeta;
  bool meta_valid = false;       // pmeta holds the current frequency set's tables
  bool near_only = false;        // only inadmissible blocks hold terms (near field of the FMM-based variant)
  // the operator's slices split into bf16 planes for GCQ_C64_SPLIT_BF16
  // products (built on first use, per block table d_bfblk)
  DevBuf bfpool, bftbuf, d_bfblk, d_bfitems, d_bfrange, d_bfrowblk, d_bfbig, d_bfmask;
  bool bf_valid = false;
  int bf_items = 0, bf_big = 0, bf_levels = 0;
  int64_t bf_bytes = 0;
  ProductGraphs graphs;
  // the operator or the frequency set changed: captured products, the
  // product's frequency tables and the bf16 copy no longer apply
  void drop_product_state() {
    graphs.clear();
    meta_valid = false;
    bf_valid = false;
    bfpool.release();   // tens of GB at 80k triangles: not kept for a rebuilt operator
    bftbuf.release();
  }
  int n_mvblocks = 0;
  int64_t storage_bytes = 0;
  int64_t last_used = 0;         // pool elements the last gcq_aca3d used (sizes the next pool)
  int last_nb = 0;               // blocks of that call's partition
  int64_t dense_bytes = 0;
};

// ---- rank model ---------------------------------------------------------------------
struct RankModel {
  bool trained = false;
  std::vector<float> params;     // 4609
  float mean[5] = {0, 0, 0, 0, 0}, stdv[5] = {1, 1, 1, 1, 1};
  DevBuf d_params;
};

// the 3D-ACA of the partition (gcq_aca3d); near_only: admissible blocks get
// no terms (the FMM-based variant compresses their M2L operators instead)
int aca3d_run(gcq_context* ctx, double tol_aca, double tol, int32_t max_freq_rank, int32_t precision,
              uint32_t flags, bool near_only, gcq_aca3d_stats* stats);
// Alg. 1 with dense slices on a batch of precomputed tensors (aca3d.hip)
// the context's side streams and fork/join events (created on first use)
int ensure_side_streams(gcq_context* ctx);
void launch_dense_aca3d(int precision, int grid, hipStream_t st, const BlockDesc3* desc, const int* qlist,
                        int nq, const int* ids, const int64_t* off, int64_t base0, const void* Cn,
                        int64_t stride, int nK, double tol, int rmax, void* pool, unsigned long long* cursor,
                        int64_t capacity, Term3* terms, int* brank, int* bstatus, int* counter);
// the 7-point rule of the far field on the reference triangle: barycentric
// points and weights (summing to 1)
void radon7(double b[7][3], double w[7]);

// ---- FMM-based 3D-ACA (gcq_fmm3d) -----------------------------------------------------
struct Fmm3D {
  bool valid = false;
  int p = 0, np3 = 0, precision = GCQ_C64, nK = 0, nfar = 0;
  int nitems = 0, nzero = 0, nleaves = 0;
  // M2L 3D-ACA of the far blocks (ctx->far_ids order): terms fstart[f] ..
  // fstart[f + 1], each a dense np3 x np3 slice and a fiber in pool
  std::vector<int> fstart, ffreq;
  std::vector<int64_t> fslice, ffiber;
  DevBuf pool;
  DevBuf d_fstart, d_fslice, d_ffiber, d_fcol, d_rowlist, d_items, d_zlist;
  // tree tables: leaves, cluster ranges, sons, parents, clusters by depth
  DevBuf d_leaves, d_clbeg, d_clend, d_son0, d_son1, d_parent, d_uplist, d_downlist, d_conj, d_kpos;
  std::vector<int> lev_start, down_start;
  // interpolation: R and L per position (leaf box), transfer into the parent per cluster
  DevBuf d_R, d_L, d_T;
  // product work buffers: permuted input, multipole and local expansions
  DevBuf Xp, W, Z;
  int64_t table_bytes = 0, m2l_bytes = 0;
  void release_work() {
    Xp.release();
    W.release();
    Z.release();
  }
};

}  // namespace gcq

struct gcq_context {
  int device = 0;
  int cus = 256;   // compute units of the device
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evm = nullptr;   // evm: a split point inside a timed region
  std::map<std::string, double> kernel_ms;
  // side streams (default priority) for concurrent work classes, created on
  // first use, and the events that fork from / join into `stream`
  hipStream_t side[3] = {nullptr, nullptr, nullptr};
  hipEvent_t evfork = nullptr, evjoin[3] = {nullptr, nullptr, nullptr};
  // launch configuration
  gcq_tuning tune = {{4, 4, 4, 4}, 8, 1, 1, 32};

  // mesh
  bool have_mesh = false;
  int n = 0;
  int64_t nv = 0;
  double c = 1.0;
  double shift[3] = {0, 0, 0};
  std::vector<double> cen, h2, area, vert;  // original order (host)

  // frequencies
  bool have_freq = false;
  int L = 0;
  std::vector<std::complex<double>> s;
  std::vector<int> rep;    // L -> representative frequency index
  std::vector<int> conj;   // L -> 1 if applied through the conjugate partner
  std::vector<int> K;      // distinct representatives, increasing
  std::vector<int> kpos;   // frequency index -> position of its representative in K

  // tree
  bool have_tree = false;
  int leaf = 0;
  double eta = 0;
  std::vector<int> perm, iperm;
  std::vector<gcq::Cluster> clusters;
  std::vector<gcq::Block> blocks;
  std::vector<int> far_ids, near_ids;       // block ids
  int depth = 0;

  // near field: element offsets of the inadmissible blocks (column-major
  // storage of one frequency) and the list of their self/near-tier entries
  std::vector<int64_t> near_off;
  int64_t near_total = 0;
  int64_t n_sing = 0;
  std::vector<int64_t> sing_off;             // element offset of each listed entry (host copy)
  gcq::DevBuf d_near_off, d_near_ids, d_sing;

  // device tables (permuted order)
  gcq::DevBuf d_cen, d_h2, d_vert, d_area, d_q64, d_c32, d_q32, d_q4, d_n64, d_n32, d_consts, d_perm, d_iperm;
  gcq::DevBuf d_blk;                         // per block: rb, re, cb, ce, flags (int32 x 5)

  gcq::HFaces H;
  gcq::Faces3D F;
  gcq::RankModel M;
  gcq::Fmm3D Mf;

  // scratch
  gcq::DevBuf scratchA, scratchB, scratchC, scratchD;
  gcq::DevBuf scratchT;                      // entry tensor of the inadmissible blocks (3D-ACA)

  gcq::Tab tab() const {
    gcq::Tab t;
    t.n = n;
    t.cen = d_cen.as<double>();
    t.h2 = d_h2.as<double>();
    t.vert = d_vert.as<double>();
    t.area = d_area.as<double>();
    t.q64 = d_q64.as<double>();
    t.c32 = d_c32.as<float>();
    t.q32 = d_q32.as<float>();
    t.q4 = reinterpret_cast<const float4*>(d_q4.as<float>());
    t.n64 = d_n64.as<double>();
    t.n32 = d_n32.as<float>();
    t.K = d_consts.as<gcq::Consts>();
    return t;
  }
};

namespace gcq {
// contexts created with device -1 hold geometry, trees and features only
#define GCQ_NEED_DEVICE(ctx) \
  do { if ((ctx)->device < 0) return ::gcq::fail(GCQ_ERR_STATE, "host-only context"); } while (0)
int check_device_ptr(gcq_context* ctx, const void* p, const char* what);
// per-device address of the staging array of gcq_assemble_slices_noalloc
// (entries.hip), resolved once per device at context creation
int noalloc_scratch_init(int device);
int timed_begin(gcq_context* ctx);
double timed_end(gcq_context* ctx, const char* name);
// a timed region in two parts split at ctx->evm (recorded by the caller on the
// context stream): the time of each part, under its name
int timed_end_split(gcq_context* ctx, const char* first, const char* second, double& ms_first,
                    double& ms_second);
inline int csize(int precision) { return precision == GCQ_C128 ? 16 : 8; }
// storage precision of a call's precision (split-bf16 products use complex64 data)
inline int storage_precision(int precision) {
  return precision == GCQ_C64_SPLIT_BF16 ? GCQ_C64 : precision;
}
}  // namespace gcq
