/*
 * gcqbem -- MI355X (gfx950) library for the frequency-domain hot path of a
 * gCQ time-domain boundary element method with H-matrix based 3D-ACA
 * (Schanz, Keshava, De Gersem, "Comparison of H-matrix- and FMM-based 3D-ACA
 * for a time-domain boundary element method", arXiv 2505.00715).
 *
 * What the library computes, all for the single-layer operator of the
 * acoustic wave equation in the Laplace domain (Sec. 2 eq. slp with the
 * kernel replaced by its transform, Sec. 3):
 *
 *   U(r, s)      = exp(-s r / c) / (4 pi r),          Re s > 0
 *   V(s)[i, j]   = int_{tau_j} U(|x_i - y|, s) dy      (piecewise-constant
 *                  basis, collocation at the centroid x_i of triangle i)
 *
 * over a closed flat-triangle surface (eq. geomapprox) and a set of complex
 * frequencies s_0..s_{L-1} (the gCQ integration points, Sec. 3 temporal
 * discretisation and App. A).  On top of the entries it builds the H-matrix
 * face of Sec. 4 (cluster tree, block cluster tree with eq. admissible, ACA
 * with QR/SVD recompression of admissible blocks, dense near field), the
 * 3D-ACA of Alg. 1 across the frequencies, and products with the compressed
 * 3D array (eq. product), including a batched iterative solve.
 *
 * Conventions
 *   - Every function returns an int status: 0 = OK, > 0 = warning, < 0 = error.
 *     On error, gcq_last_error() gives a message (thread-local, valid until the
 *     next call on the same thread).  No C++ exception crosses this boundary.
 *   - Indices are 0-based and refer to the caller's triangle order; the
 *     library's cluster permutation is internal.
 *   - Complex numbers are interleaved (re, im): gcq_c128 for double, pairs of
 *     float for single precision.
 *   - "host" arguments are plain host pointers; the library copies what it
 *     needs before returning and never keeps them.  "device" arguments are
 *     device pointers owned by the caller (for example torch tensors on the
 *     same GPU); the library checks that they are device memory, never frees
 *     them, and only accesses them inside the call's stream work.
 *   - All device work is enqueued on the context's stream.  Calls that return
 *     host statistics synchronise that stream; the products do not.
 *   - Call order: upload_mesh -> set_frequencies -> build_cluster_tree ->
 *     {aca_blocks | aca3d} -> products / solve.  A call made too early returns
 *     GCQ_ERR_STATE.  Uploading a mesh or frequencies invalidates everything
 *     built on them.
 */
#ifndef GCQBEM_H
#define GCQBEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GCQ_API __attribute__((visibility("default")))

typedef struct gcq_context gcq_context;

typedef struct {
  double re, im;
} gcq_c128;

/* Arithmetic of a call.
 *   GCQ_C128: complex128 throughout.
 *   GCQ_C64:  complex64 far-field entries, low-rank factors and products with
 *             float accumulation; the self and near-singular quadrature and
 *             every stopping-criterion norm stay in float64.
 *   GCQ_C64_SPLIT_BF16: products only (gcq_compressed_matvec in
 *             GCQ_PER_FREQUENCY mode, gcq_solve) with an operator built at
 *             GCQ_C64, complex64 vectors, on the bf16 matrix cores with float
 *             accumulation: the operator's float values a are split into two
 *             bf16 planes (ha = bf16(a), la = bf16(a - ha); a fixed relative
 *             perturbation <= 2^-18 of the operator), the vectors' values x
 *             into three (hx, mx, lx; <= 2^-27), and each real product is
 *             ha hx + ha mx + ha lx + la hx + la mx, which is linear in x up
 *             to 2^-26 |a| |x| (so GMRES converges as with complex64).  The
 *             split copy of the operator (as many bytes as its complex64
 *             slices) is made on the first such product and kept with the
 *             operator. */
enum { GCQ_C128 = 0, GCQ_C64 = 1, GCQ_C64_SPLIT_BF16 = 2 };

/* Product modes of gcq_compressed_matvec.
 *   GCQ_PER_FREQUENCY: Y[k] = V(s_k) X[k] for every frequency k, V(s_k)
 *                      the 3D-ACA approximant.
 *   GCQ_WEIGHTED_SUM:  y = sum_k V(s_k) X[k] (eq. product: the frequency sum
 *                      is taken per slice before the spatial product).
 *   GCQ_PLAIN_H:       Y[k] = V_H(s_k) X[k] with the per-frequency H-matrices
 *                      of gcq_aca_blocks (no frequency compression). */
enum { GCQ_PER_FREQUENCY = 0, GCQ_WEIGHTED_SUM = 1, GCQ_PLAIN_H = 2 };

/* Status codes. */
enum {
  GCQ_OK = 0,
  GCQ_NOT_CONVERGED = 1, /* solve: some system missed the tolerance            */
  GCQ_RANK_CAPPED = 2,   /* aca_blocks / aca3d: some block hit its rank limit   */
  GCQ_ERR_ARG = -1,      /* invalid argument (null, range, host-vs-device)     */
  GCQ_ERR_NOMEM = -2,    /* device allocation failed                           */
  GCQ_ERR_HIP = -3,      /* HIP runtime error                                  */
  GCQ_ERR_STATE = -4,    /* call order violated                                */
  GCQ_ERR_NUMERIC = -5,  /* degenerate geometry or non-finite data             */
  GCQ_ERR_UNSUPPORTED = -6
};

/* Flags of gcq_aca_blocks. */
enum {
  GCQ_FLAG_RECOMPRESS = 1u,      /* QR/SVD recompression after ACA (Sec. 4)          */
  GCQ_FLAG_USE_PREDICTOR = 2u,   /* size work tiles from the trained rank model      */
  GCQ_FLAG_PER_FREQ_LAUNCH = 4u, /* one launch per frequency, no batching (baseline)  */
  GCQ_FLAG_DOUBLE_LAYER = 8u     /* faces of the double layer K (Sec. 2 eq. dlp) with
                                    the entries of gcq_assemble_dlp_slices; not with
                                    GCQ_FLAG_USE_PREDICTOR (GCQ_ERR_ARG)            */
};

/* Launch configuration (gcq_set_tuning / gcq_get_tuning).
 *   aca3d_waves[c]: wave64s that work together on one admissible block in
 *     gcq_aca3d, for blocks with |I| + |J| <= 160, <= 320, <= 640 and > 640
 *     (c = 0..3); each 1, 2, 4 or 8.  Default {4, 4, 4, 4}.  Blocks whose
 *     accepted slices outgrow the group's on-chip storage are redone with
 *     twice the waves.
 *   aca3d_stack_slices: initial reservation of an admissible block's stacked
 *     slice factors, in slices of full ACA rank (1..64, default 8); a block
 *     that needs more moves its stack to a reservation twice as large.
 *   aca_waves, product_graph, product_cols_per_wave: see the fields.
 * Results do not depend on the configuration beyond rounding order. */
typedef struct {
  int32_t aca3d_waves[4];
  int32_t aca3d_stack_slices;
  int32_t aca_waves;           /* wave64s per (block, frequency) pair in gcq_aca_blocks:
                                  1, 2 or 4 (default 1) */
  int32_t product_graph;       /* 1 (default): gcq_compressed_matvec and gcq_solve replay
                                  the per-frequency product as a captured HIP graph;
                                  0: plain launches */
  int32_t product_cols_per_wave; /* frequency columns a wave64 of the split-bf16
                                  product owns: 32 (default; 8 waves per workgroup)
                                  or 64 (4 waves; each operator fragment serves two
                                  32-column tiles) */
} gcq_tuning;

typedef struct {
  int32_t n_clusters;
  int32_t n_leaves;
  int32_t depth;       /* levels below the root                       */
  int32_t n_blocks;    /* leaves of the block cluster tree            */
  int32_t n_far;       /* admissible blocks                           */
  int32_t n_near;      /* inadmissible (dense) blocks                 */
  int64_t far_dims;    /* sum over far blocks of |I| + |J|            */
  int64_t near_entries;/* sum over near blocks of |I| |J|             */
} gcq_tree_info;

typedef struct {
  int64_t n_pairs;          /* (far block, frequency) pairs approximated       */
  int64_t aca_rank_sum;     /* sum of ACA ranks                                */
  int64_t rank_sum;         /* sum of ranks after recompression                */
  int32_t rank_max;
  int32_t n_capped;         /* pairs that hit max_rank                         */
  int64_t n_overflow;       /* pairs re-run because their tile was too small   */
  int64_t entries;          /* kernel entries evaluated (rows + columns)       */
  int64_t storage_bytes;    /* compressed far field + dense near field         */
  double device_ms;         /* device time of the call                         */
} gcq_aca_stats;

typedef struct {
  int32_t n_blocks;
  int32_t rank_min, rank_max; /* frequency ranks r_b over blocks              */
  double rank_mean;
  int32_t n_capped;           /* blocks that reached max_freq_rank            */
  int64_t slice_rank_sum;     /* sum over far slices of their ACA rank        */
  int64_t storage_bytes;      /* slices + fibers                               */
  double compression_rate;    /* storage / dense storage of all |K| matrices  */
  double device_ms;
  /* work of the admissible blocks' kernel, counted on the device: kernel
   * entries evaluated (slice rows and columns, fibers), and the algorithmic
   * floating-point operations of the method's steps (20 per far-field
   * quadrature point, 8 per complex multiply-add of the residual corrections,
   * pivot expansions, Gram and slice inner products, fibers) */
  int64_t far_entries;
  double far_flops;
  double far_ms;              /* device time of the admissible blocks' kernels */
} gcq_aca3d_stats;

typedef struct {
  int32_t n_systems;
  int32_t n_converged;
  int32_t iters_max;
  double resid_max;           /* max over systems of |b - A x| / |b|          */
  double device_ms;
} gcq_solve_stats;

typedef struct {
  int32_t epochs;
  int32_t batch;
  float lr, beta1, beta2, eps;
  uint64_t seed;              /* shuffling and initialisation                  */
} gcq_train_cfg;

typedef struct {
  float loss_first, loss_last; /* mean loss of the first and last epoch        */
  double device_ms;
} gcq_train_stats;

/* ---- context --------------------------------------------------------------
 * gcq_create: context on HIP device `device`, enqueuing on `hip_stream`
 *   (a hipStream_t; NULL = the device's null stream).  *out receives the
 *   context; the caller releases it with gcq_destroy, which frees every device
 *   allocation the library made for it. */
GCQ_API int gcq_create(int device, void* hip_stream, gcq_context** out);
GCQ_API int gcq_destroy(gcq_context* ctx);
GCQ_API const char* gcq_last_error(void);
/* Device time (ms) of the library's most recent kernel of the named kind
 * ("aca", "recompress", "aca3d", "matvec", ...) as measured with HIP events,
 * or -1 if none. */
GCQ_API double gcq_kernel_ms(gcq_context* ctx, const char* name);

/* gcq_set_tuning / gcq_get_tuning: replace / read the launch configuration
 *   of the context (host struct, copied).  GCQ_ERR_ARG on values out of range;
 *   the configuration is then unchanged. */
GCQ_API int gcq_set_tuning(gcq_context* ctx, const gcq_tuning* tuning);
GCQ_API int gcq_get_tuning(gcq_context* ctx, gcq_tuning* tuning);

/* ---- geometry and frequencies (Sec. 3; Sec. 2) ------------------------------
 * gcq_upload_mesh: host xyz (n_vertices x 3 doubles, row-major) and tri
 *   (n_triangles x 3 int32 vertex ids, outward orientation) of Gamma_h
 *   (eq. geomapprox); wave speed c > 0.  Builds the panel tables on the device
 *   (centroids, longest edges, 7-point quadrature of each triangle).
 *   GCQ_ERR_NUMERIC for a zero-area triangle or non-finite coordinates. */
GCQ_API int gcq_upload_mesh(gcq_context* ctx, const double* xyz, int64_t n_vertices,
                            const int32_t* tri, int64_t n_triangles, double wave_speed);

/* gcq_set_frequencies: host array of n_freq complex frequencies s_k (the
 *   points at which the 3D array of Sec. 3 is sampled); Re s_k > 0 is
 *   required (GCQ_ERR_ARG otherwise).  With use_conjugate_symmetry != 0, a
 *   frequency k > n_freq/2 whose value is the conjugate of s_{n_freq-k} is
 *   represented by that partner (V(conj s) = conj V(s)), so only the set
 *   K = {0..n_freq/2} is ever approximated (Sec. 5.1; App. A). */
GCQ_API int gcq_set_frequencies(gcq_context* ctx, const gcq_c128* s, int32_t n_freq,
                                int32_t use_conjugate_symmetry);

/* gcq_contour: points s_l and weights w_l, l = 1..n_points, of the gCQ
 *   contour quadrature of App. A (no context, host arrays of n_points
 *   complex doubles, owned by the caller).  q = stage_ratio * dt_max / dt_min
 *   (stage_ratio = 1 for implicit Euler, 5 max|lambda(A)| / min|lambda(A)| for
 *   a Runge-Kutta method of several stages), elliptic modulus
 *   k = (q - sqrt(2q-1)) / (q + sqrt(2q-1)), K = K(k^2), K' = K(1 - k^2),
 *   sigma_l = -K + (l - 1/2) 4K / n_points + i K'/2, s_l = gamma(sigma_l),
 *   w_l = 4K / (2 pi i n_points) gamma'(sigma_l) (the appendix's map gamma;
 *   the weight's denominator reads 2 pi i n_points where the printed formula
 *   is garbled).  The contour is traversed clockwise as Re sigma grows:
 *   sum_l w_l f(s_l) approximates -(1 / 2 pi i) times the counter-clockwise
 *   integral of f.  The points come in conjugate pairs s_{n+1-l} = conj(s_l);
 *   for odd n_points the middle point is real.  All points have Re s > 0.
 *   The curve crosses the real axis at 0 and 2 / dt_min: for a Runge-Kutta
 *   method of several stages pass dt_min / x* and dt_max / x*, x* the end of
 *   the interval (0, x*) on which the method's stability function exceeds 1
 *   in modulus (6 for 2-stage Radau IIA), so that the states of the stepping
 *   do not grow on the contour.
 *   GCQ_ERR_ARG for n_points < 1, NULL arrays, dt_min <= 0, dt_max < dt_min,
 *   stage_ratio < 1, or q <= 1 (constant steps: the appendix perturbs q). */
GCQ_API int gcq_contour(int32_t n_points, double dt_min, double dt_max, double stage_ratio,
                        gcq_c128* s, gcq_c128* w);

/* gcq_contour_steps: the arguments (dt_min', dt_max', stage_ratio) of
 *   gcq_contour for an m-stage Runge-Kutta method with Butcher matrix A (host,
 *   m x m doubles, row-major, 1 <= m <= 4) and steps between dt_min and dt_max
 *   (App. A, q = 5 dt_max max|lambda(A)| / (dt_min min|lambda(A)|)): for m > 1,
 *   args = (dt_min / x*, dt_max / x*, 5 max|lambda(A)| / min|lambda(A)|) with x*
 *   the end of the interval (0, x*) of the positive real axis on which the
 *   stability function R(x) = e_m^T (I - x A)^{-1} 1 exceeds 1 in modulus (the
 *   contour then crosses the real axis at 2 x* / dt_min); for m = 1,
 *   (dt_min A, dt_max A, 1).  args: host, 3 doubles.  GCQ_ERR_ARG for invalid
 *   sizes or steps, a singular A, or no such interval within (0, 200];
 *   GCQ_ERR_NUMERIC when A is not diagonalisable. */
GCQ_API int gcq_contour_steps(const double* A, int32_t m, double dt_min, double dt_max, double* args);

/* gcq_contour_points: the number N_Q of contour points for n_steps >= 2 steps
 *   of a method with `stages` stages (Sec. 3, cost estimate after
 *   eq. gcq_formula, and App. A): N log N for one stage, N (log N)^2 for more,
 *   natural logarithm, as twice the rounded half (the points pair up by
 *   conjugation; the half is what Sec. 5.1 tabulates).  GCQ_ERR_ARG for
 *   n_steps < 2, stages < 1 or a count beyond int32. */
GCQ_API int gcq_contour_points(int32_t n_steps, int32_t stages, int32_t* n_points);

/* gcq_gcq_convolve: the forward gCQ convolution f = V * q (Sec. 3: the first
 *   step, eq. gCQ_xn and eq. gcq_formula) for an m-stage Runge-Kutta method
 *   with Butcher matrix A (host, m x m doubles, row-major, 1 <= m <= 4, with
 *   b^T A^{-1} = (0, .., 0, 1) as for Radau IIA; implicit Euler is m = 1,
 *   A = (1)) on the operator gcq_aca3d built at `precision`, for n_steps steps
 *   of sizes dt[0..n_steps) (host array; variable steps are what the
 *   generalised scheme is for).  The context's frequency set must be [step
 *   points, contour points]: among its first n_step_points frequencies are the
 *   values lam_e / dt_n for every eigenvalue lam_e of A^{-1} and every step
 *   (1/dt_n for implicit Euler; matched to 1e-10 relative, GCQ_ERR_STATE
 *   otherwise), the remaining NQ = n_freq - n_step_points are the contour
 *   points, whose weights w (host, NQ complex doubles, as gcq_contour returns
 *   them) are passed here.  One step point and odd NQ give the pairing
 *   k <-> n_freq - k that conjugate symmetry uses; more step points need a set
 *   without it.  With A^{-1} = P diag(lam) P^{-1} and M_l(dt) = (I - dt s_l A)^{-1},
 *   per step n:
 *     x_{n-1}(s_l) = M_l(dt_{n-1}) ((x_{n-2}(s_l))_m 1 + dt_{n-1} A q_{n-1}), x_0 = 0,
 *     f_n = P diag(V(lam_e / dt_n)) P^{-1} q_n + sum_l V(s_l) w_l (x_{n-1}(s_l))_m M_l(dt_n) 1
 *   (per stage one product over the set, summed over its columns: the stage
 *   value is the real part).  Q (input) and F (output) are device arrays of
 *   n_steps x m x n_triangles doubles (step, stage, triangle order), checked
 *   to be device memory (GCQ_ERR_ARG otherwise).  The
 *   state (NQ x n complex doubles: only the last stage of x enters) and the
 *   product's columns are allocated for the call; returns after the last step.
 *   GCQ_ERR_ARG for a singular A, GCQ_ERR_NUMERIC when A^{-1} is not
 *   diagonalisable with distinct eigenvalues. */
GCQ_API int gcq_gcq_convolve(gcq_context* ctx, const double* A, int32_t m, const double* dt,
                             int32_t n_steps, int32_t n_step_points, const gcq_c128* w,
                             int32_t precision, const double* Q, double* F);

/* gcq_gcq_solve: the same scheme with (f)_n given and the density unknown
 *   (eq. gcq_formula, solved step by step for q_n): per step the history
 *   h = sum_l V(s_l) w_l (x_{n-1}(s_l))_m M_l(dt_n) 1 of the densities found so
 *   far, then V((dt_n A)^{-1}) q_n = f_n - h, decoupled by P into the systems
 *   V(lam_e / dt_n) y_e = (P^{-1} (f_n - h))_e solved by GMRES (gcq_solve's
 *   batched solver; the other frequencies' systems have zero right-hand sides
 *   and end at once), q_n = P y.  F (input) and Q (output): device doubles,
 *   n_steps x m x n_triangles.  rtol, max_iter, restart as in gcq_solve;
 *   *iters_max (may be NULL) receives the largest iteration count of a step.
 *   Returns GCQ_NOT_CONVERGED (after the last step) if the solve of some step
 *   ended above rtol: its density, inaccurate, then also entered the history
 *   of every later step.  F and Q must be device memory (GCQ_ERR_ARG
 *   otherwise), as for gcq_gcq_convolve. */
GCQ_API int gcq_gcq_solve(gcq_context* ctx, const double* A, int32_t m, const double* dt,
                          int32_t n_steps, int32_t n_step_points, const gcq_c128* w,
                          int32_t precision, const double* F, double* Q, double rtol,
                          int32_t max_iter, int32_t restart, int32_t* iters_max);

/* gcq_build_cluster_tree: cluster tree and block cluster tree of Sec. 4
 *   (eq. admissible with parameter eta > 0, leaves of at most leaf_size
 *   triangles).  info may be NULL. */
GCQ_API int gcq_build_cluster_tree(gcq_context* ctx, int32_t leaf_size, double eta,
                                   gcq_tree_info* info);

/* gcq_upload_cluster_tree: a cluster tree and block cluster tree made by the
 *   caller (Sec. 4: cluster tree, block cluster tree, eq. admissible), used
 *   instead of gcq_build_cluster_tree's own, so that another implementation's
 *   partition (an oracle's, a PCA split as the paper's) can be injected.  All
 *   arrays are host memory, copied:
 *     perm (n_triangles): cluster position -> caller's triangle index, a
 *       permutation;
 *     cl_begin, cl_end (n_clusters): each cluster is positions [begin, end),
 *       non-empty; cluster 0 is the root [0, n_triangles);
 *     cl_son (2 x n_clusters): the two sons of a cluster, which split its range
 *       in two (first son first) and have larger indices than it, or (-1, -1)
 *       for a leaf; every cluster but the root is the son of exactly one;
 *     blk_row, blk_col, blk_admissible (n_blocks): the leaves of the block
 *       tree as cluster pairs and their admissibility (0 or 1).  They must be
 *       the leaves of a block tree over this cluster tree: from (root, root),
 *       each pair that is not a block is split through the sons of the
 *       clusters that have them, and every block must be reached; so the blocks
 *       cover every (row, column) pair exactly once.  An admissible block's
 *       clusters need vertex boxes at positive distance (eq. admissible with
 *       some eta); the library does not test the eta condition itself.
 *   The blocks keep the caller's order (block indices of gcq_get_tree,
 *   gcq_get_block_factors and gcq_get_aca3d_block are positions in it).
 *   info may be NULL.  GCQ_ERR_ARG for any violation (nothing is changed);
 *   GCQ_ERR_STATE without a mesh.  Like gcq_build_cluster_tree, it
 *   invalidates faces and operators built on an earlier tree. */
GCQ_API int gcq_upload_cluster_tree(gcq_context* ctx, const int32_t* perm, int32_t n_clusters,
                                    const int32_t* cl_begin, const int32_t* cl_end,
                                    const int32_t* cl_son, int32_t n_blocks, const int32_t* blk_row,
                                    const int32_t* blk_col, const uint8_t* blk_admissible,
                                    gcq_tree_info* info);

/* gcq_trim: releases the device memory the context keeps between calls for
 *   its working buffers (ACA workspaces, entry tensors, tables), which the
 *   next call allocates again; with release_faces != 0 also the per-frequency
 *   H-matrices of gcq_aca_blocks (GCQ_PLAIN_H products then need a new
 *   gcq_aca_blocks).  The products' buffers and the split-bf16 copy of the
 *   operator are released too (the next product makes them again); the
 *   3D-ACA operator itself stays.  Synchronises the context's streams. */
GCQ_API int gcq_trim(gcq_context* ctx, int32_t release_faces);

/* gcq_get_tree: copies the partition to host arrays: perm (n_triangles:
 *   internal position -> caller index) and blocks (n_blocks x 5 int32:
 *   row_begin, row_end, col_begin, col_end in internal positions, admissible),
 *   in depth-first order (an uploaded tree: the caller's block order).
 *   Either pointer may be NULL. */
GCQ_API int gcq_get_tree(gcq_context* ctx, int32_t* perm, int32_t* blocks);

/* ---- entries (Sec. 3) -----------------------------------------------------
 * gcq_assemble_slices: dense entries V(s_f)[rows[a], cols[b]] for the host
 *   index lists rows (n_rows), cols (n_cols) and frequency indices freq_idx
 *   (n_fidx, each in 0..n_freq-1).  out_dev (device, caller-owned) receives
 *   n_fidx x n_cols x n_rows complex values, rows fastest (column-major per
 *   slice): complex128 for GCQ_C128, complex64 for GCQ_C64 (far entries then
 *   computed in float; self and near entries always in double). */
GCQ_API int gcq_assemble_slices(gcq_context* ctx, const int32_t* rows, int64_t n_rows,
                                const int32_t* cols, int64_t n_cols, const int32_t* freq_idx,
                                int32_t n_fidx, int32_t precision, void* out_dev);

/* gcq_assemble_slices_noalloc: gcq_assemble_slices for callers that cannot
 *   allocate device memory (code under HIP graph capture, serving loops,
 *   harnesses that forbid hipMalloc): same arguments, layout and results, but
 *   the permuted index lists and the frequencies are staged in a fixed 8 MiB
 *   array of each device (one per GPU for the life of the process) instead of
 *   the context's buffers, and the call allocates nothing, records no timing
 *   and returns without synchronising.  A request needs
 *   ceil256(4 n_rows) + ceil256(4 n_cols) + 16 n_fidx bytes of staging
 *   (ceil256 rounds up to a multiple of 256); GCQ_ERR_ARG above 8 MiB.  Every
 *   call on a GPU shares that GPU's array: calls that overlap on one GPU (two
 *   contexts or streams, or a second call while a first one's kernel has not
 *   started) race; every part of the array a call reads is written by that
 *   call first, so nothing needs clearing between calls. */
GCQ_API int gcq_assemble_slices_noalloc(gcq_context* ctx, const int32_t* rows, int64_t n_rows,
                                        const int32_t* cols, int64_t n_cols, const int32_t* freq_idx,
                                        int32_t n_fidx, int32_t precision, void* out_dev);

/* gcq_assemble_dlp_slices: dense double-layer entries K(s_f)[rows[a], cols[b]]
 *   (Sec. 2, eq. dlp, transformed as in Sec. 3): the integral over panel
 *   cols[b] of the normal derivative in y (outward unit normal of the panel,
 *   from its vertex order) of exp(-s r / c) / (4 pi r), collocated at the
 *   centroid of panel rows[a] with piecewise-constant densities; self entries
 *   are 0 (flat panels), near and far tiers as in gcq_assemble_slices (near
 *   always in float64).  Arguments, layout and errors as gcq_assemble_slices. */
GCQ_API int gcq_assemble_dlp_slices(gcq_context* ctx, const int32_t* rows, int64_t n_rows,
                                    const int32_t* cols, int64_t n_cols, const int32_t* freq_idx,
                                    int32_t n_fidx, int32_t precision, void* out_dev);

/* ---- H-matrix faces per frequency (Sec. 4) --------------------------------
 * gcq_aca_blocks: ACA (partial pivoting, relative tolerance tol, at most
 *   max_rank terms) of every admissible block at every frequency of K (or of
 *   the n_fidx listed representatives when freq_idx != NULL), followed by
 *   QR/SVD recompression when GCQ_FLAG_RECOMPRESS is set; near blocks are
 *   assembled densely.  The result is kept in the context for GCQ_PLAIN_H
 *   products and gcq_get_block_factors.  Returns GCQ_RANK_CAPPED if some pair
 *   reached max_rank.  stats may be NULL. */
GCQ_API int gcq_aca_blocks(gcq_context* ctx, const int32_t* freq_idx, int32_t n_fidx,
                           double tol, int32_t max_rank, int32_t precision, uint32_t flags,
                           gcq_aca_stats* stats);

/* gcq_aca_ranks: the ranks (after recompression) of every (admissible block,
 *   frequency) pair of the last gcq_aca_blocks, into the host array ranks of
 *   n = n_far x n_slots values, [far block in depth-first order][frequency slot
 *   in the call's order] (the layout of gcq_rank_features).  GCQ_ERR_ARG when n
 *   differs; GCQ_ERR_STATE before gcq_aca_blocks. */
GCQ_API int gcq_aca_ranks(gcq_context* ctx, int32_t* ranks, int64_t n);

/* gcq_get_block_factors: host copy of the factors of admissible block `block`
 *   (index into the depth-first block list) at representative frequency
 *   `freq`: U (|I| x rank) and V (|J| x rank), column-major complex128, rows
 *   in internal order of the block's clusters, with A_b(s) ~ U V^H.  Buffers
 *   must hold cap columns; *rank receives the rank (GCQ_ERR_ARG if > cap). */
GCQ_API int gcq_get_block_factors(gcq_context* ctx, int32_t block, int32_t freq, gcq_c128* U,
                                  gcq_c128* V, int32_t cap, int32_t* rank);

/* ---- 3D-ACA (Sec. 4, Alg. 1, eq. norm) ------------------------------------
 * gcq_aca3d: per block of the partition, the 3D-ACA over the frequencies of K
 *   with slice tolerance tol_aca (ACA + recompression of far slices) and
 *   frequency tolerance tol, at most max_freq_rank terms per block.  flags:
 *   GCQ_FLAG_DOUBLE_LAYER compresses the double layer K(s) (entries of
 *   gcq_assemble_dlp_slices) instead of V(s); the products and the gCQ
 *   stepping then apply K.  Other flag bits are ignored. */
GCQ_API int gcq_aca3d(gcq_context* ctx, double tol_aca, double tol, int32_t max_freq_rank,
                      int32_t precision, uint32_t flags, gcq_aca3d_stats* stats);

/* gcq_get_aca3d_block: host copy of block `block`'s 3D-ACA: *rank terms,
 *   freqs (rank positions in K), fibers (rank x |K| complex128) and the dense
 *   expansion of each slice (rank x |J| x |I| complex128, column-major per
 *   slice, internal order).  Buffers must hold cap terms. */
GCQ_API int gcq_get_aca3d_block(gcq_context* ctx, int32_t block, int32_t cap, int32_t* rank,
                                int32_t* freqs, gcq_c128* fibers, gcq_c128* slices);

/* gcq_aca3d_ranks: per block of the partition (depth-first order) the number
 *   of terms of its 3D-ACA (Alg. 1) into terms[b], and for an admissible block
 *   the sum of its slices' ranks (the stacked columns of Ubar and Vbar that the
 *   products of eq. product contract over) into columns[b]; 0 for an
 *   inadmissible block, whose slices are dense.  Host arrays of n = number of
 *   blocks values (GCQ_ERR_ARG otherwise); GCQ_ERR_STATE before gcq_aca3d. */
GCQ_API int gcq_aca3d_ranks(gcq_context* ctx, int32_t* terms, int32_t* columns, int64_t n);

/* ---- FMM-based 3D-ACA (Sec. 4: the face by a black-box FMM, eq. cheb) --------
 * gcq_fmm3d: the FMM-based variant of the 3D-ACA on the context's partition.
 *   The far field of an admissible block (X, Y) is the Chebyshev
 *   interpolation of the kernel in both clusters' boxes (eq. cheb):
 *     A_XY(s) ~ L_X K_XY(s) R_Y^T,  L_X[i, n] = S_X(x_i, x_n),
 *     R_Y[j, m] = sum_q w_jq S_Y(y_jq, y_m) (the far 7-point rule),
 *     K_XY(s)[n, m] = exp(-s r / c) / (4 pi r), r = |x_n - y_m|,
 *   with `order` Chebyshev nodes (the zeros of T_order) per dimension in each
 *   cluster's vertex box (a half-width below 1e-3 of the box's largest is
 *   raised to that), nodes numbered n = a_x + p a_y + p^2 a_z.  Only the M2L
 *   operators K_XY(s) depend on the frequency: Alg. 1 (eq. norm, tolerance
 *   tol, at most max_freq_rank terms) compresses each admissible block's
 *   tensor [K_XY(s_k)]_k over the frequencies of K with dense p^3 x p^3
 *   slices; inadmissible blocks as in gcq_aca3d.  order 1..6; precision
 *   GCQ_C128 or GCQ_C64.  The context's 3D-ACA operator is replaced: until
 *   gcq_aca3d runs again, gcq_compressed_matvec, gcq_solve, gcq_sample_rows and
 *   the gCQ calls return GCQ_ERR_STATE.  stats may be NULL. */
typedef struct {
  int32_t n_far;          /* admissible blocks, i.e. M2L tensors */
  int32_t rank_max;       /* most terms of an M2L tensor */
  double rank_mean;       /* mean terms of the M2L tensors */
  int32_t n_capped;       /* M2L tensors that reached max_freq_rank */
  int64_t storage_bytes;  /* M2L slices and fibers, interpolation and transfer
                             tables, near-field slices and fibers */
  double device_ms;       /* device time of the build */
  double m2l_ms;          /* of which the M2L entries and their 3D-ACA */
} gcq_fmm3d_stats;
GCQ_API int gcq_fmm3d(gcq_context* ctx, int32_t order, double tol, int32_t max_freq_rank,
                      int32_t precision, gcq_fmm3d_stats* stats);

/* gcq_fmm3d_matvec: Y[k] = V~(s_k) X[k] for every frequency with the operator
 *   of gcq_fmm3d: the near blocks as gcq_compressed_matvec (GCQ_PER_FREQUENCY)
 *   applies them, then the far field added by the multi-level evaluation
 *   P2M (R^T at the leaves), M2M, M2L (sum_d f_d[k] H_d), L2L, L2P (L at the
 *   leaves), which equals the single-level form above up to rounding (a
 *   parent's Lagrange polynomials are interpolated exactly by a son's nodes).
 *   X_dev, Y_dev: device arrays of L x n complex values in gcq_fmm3d's
 *   precision, frequency-major, caller's triangle order (GCQ_ERR_ARG for
 *   host memory); GCQ_ERR_STATE before gcq_fmm3d or after a gcq_aca3d. */
GCQ_API int gcq_fmm3d_matvec(gcq_context* ctx, const void* X_dev, void* Y_dev);

/* gcq_get_fmm3d_block: host copy of admissible block `block`'s M2L 3D-ACA:
 *   *rank terms, freqs (positions in K), fibers (rank x |K| complex128) and
 *   slices (rank x p^3 x p^3 complex128, column-major: entry (n, m) at
 *   m p^3 + n, n a node of the row cluster's box, m of the column
 *   cluster's).  Buffers hold cap terms (GCQ_ERR_ARG otherwise); freqs,
 *   fibers, slices may be NULL. */
GCQ_API int gcq_get_fmm3d_block(gcq_context* ctx, int32_t block, int32_t cap, int32_t* rank,
                                int32_t* freqs, gcq_c128* fibers, gcq_c128* slices);

/* gcq_sample_rows: rows of the compressed 3D array at frequency `freq`
 *   (0..n_freq-1): out[a][j] = V~(s_freq)[rows[a], j] for every column j,
 *   V~(s) = sum_b sum_d f_{b,d}(s) H_{b,d} the approximant of Alg. 1 that the
 *   products of eq. product apply (conjugated for a frequency represented by
 *   its conjugate partner).  rows: host, n_rows caller indices (repeats
 *   allowed); out_dev: device, n_rows x n_triangles complex values, row-major,
 *   columns in the caller's order, complex128 or complex64 as the operator was
 *   built; caller-owned.  Returns after the rows are written.  GCQ_ERR_STATE
 *   before gcq_aca3d; GCQ_ERR_ARG for indices out of range or host memory
 *   as out_dev. */
GCQ_API int gcq_sample_rows(gcq_context* ctx, const int32_t* rows, int32_t n_rows, int32_t freq,
                            void* out_dev);

/* ---- products (eq. product) -----------------------------------------------
 * gcq_compressed_matvec: X_dev, Y_dev are device arrays of n_cols vectors of
 *   length n_triangles, vector-major (torch shape (n_cols, n), contiguous);
 *   complex128 for GCQ_C128, complex64 for GCQ_C64 and GCQ_C64_SPLIT_BF16
 *   (GCQ_PER_FREQUENCY only; GCQ_ERR_UNSUPPORTED for the other modes).
 *   n_cols must equal n_freq.  For GCQ_WEIGHTED_SUM, Y_dev holds one vector.
 *   Enqueued on the context stream without synchronisation. */
GCQ_API int gcq_compressed_matvec(gcq_context* ctx, int32_t mode, int32_t precision,
                                  const void* X_dev, void* Y_dev, int32_t n_cols);

/* ---- batched solve ---------------------------------------------------------
 * gcq_solve: solves V(s_k) x_k = b_k for every frequency k at once with
 *   restarted GMRES(restart) on the 3D-ACA operator, orthogonalisation in
 *   float64 (classical Gram-Schmidt twice), until |b - A x| <= rtol |b| or
 *   max_iter iterations.  B_dev, X_dev: complex128 device arrays shaped like
 *   the products' X.  The product inside uses `precision` (GCQ_C64_SPLIT_BF16
 *   with an operator built at GCQ_C64).  With product_graph set (default)
 *   each Arnoldi step runs as a replayed graph, and a 32-column frequency tile
 *   whose systems all have residual estimates below rtol / 2 is left out of
 *   the split-bf16 products; every system's update uses the steps its tile
 *   computed (likewise with the graph off).  Returns GCQ_NOT_CONVERGED if some
 *   system missed the tolerance. */
GCQ_API int gcq_solve(gcq_context* ctx, const void* B_dev, void* X_dev, double rtol,
                      int32_t max_iter, int32_t restart, int32_t precision,
                      gcq_solve_stats* stats);

/* ---- learned rank predictor -----------------------------------------------
 * The network (5 -> 64 -> 64 -> 1, tanh, float) maps standardised features of
 * a (far block, frequency) pair to log(1 + ACA rank).  Parameters are laid
 * out W1(64x5) b1(64) W2(64x64) b2(64) W3(1x64) b3(1), row-major; 4609 floats.
 *
 * gcq_rank_features: host features (n_far x n_fidx x 5 floats, unstandardised)
 *   of every admissible block at the listed representatives:
 *   [diam |s|/c, dist Re(s)/c, dist |Im s|/c, log2|I|, log2|J|].
 * gcq_rank_model_train: trains on m host samples (feat m x 5, unstandardised;
 *   target m floats = log(1 + rank)) with the library's forward, backward and
 *   Adam kernels; standardisation is fitted on the training set.
 * gcq_rank_model_grad: one forward/backward pass at the current parameters
 *   on m host samples (already standardised); writes the mean loss and the
 *   gradient (4609 floats) to host memory.
 * gcq_rank_model_predict: predicted log(1 + rank) for m host samples.
 * gcq_rank_model_get / set: host copy of parameters (4609 floats) and of the
 *   standardisation (mean[5], std[5]; either pointer may be NULL). */
GCQ_API int gcq_rank_features(gcq_context* ctx, const int32_t* freq_idx, int32_t n_fidx,
                              float* feat);
GCQ_API int gcq_rank_model_train(gcq_context* ctx, const float* feat, const float* target,
                                 int64_t m, const gcq_train_cfg* cfg, gcq_train_stats* stats);
GCQ_API int gcq_rank_model_grad(gcq_context* ctx, const float* feat_std, const float* target,
                                int64_t m, float* loss, float* grad);
GCQ_API int gcq_rank_model_predict(gcq_context* ctx, const float* feat, int64_t m,
                                   float* out);
GCQ_API int gcq_rank_model_get(gcq_context* ctx, float* params, float* mean, float* std);
GCQ_API int gcq_rank_model_set(gcq_context* ctx, const float* params, const float* mean,
                               const float* std);

#ifdef __cplusplus
}
#endif
#endif /* GCQBEM_H */
