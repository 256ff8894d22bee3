/*
 * h2.h -- C-ABI of an MI355X (gfx950) implementation of adaptive
 * H^2-matrix multiplication Z <- Z + X Y (S. Boerm, "Adaptive fast
 * multiplication of H^2-matrices", arXiv 2309.09061).
 *
 * The operation is split as in the paper's Introduction into
 *   phase 1 (h2_mul_intermediate): compressed induced row and column cluster
 *     bases (Section 4, Figure "induced_basis") with block-relative error
 *     control (Section 5), and the intermediate product G on the product
 *     block tree T^XY (Section 6, opening definition);
 *   phase 2 (h2_recompress): coarsening of G into the prescribed block tree
 *     T_IK with adaptive nested isometric bases (Section 6, Figures
 *     "match_column" and "basis").
 *
 * Conventions common to every call:
 *  - Status codes are returned; nothing throws across the ABI.  On error the
 *    output handles are left untouched (set to NULL) and a thread-local
 *    message is available from h2_last_error().
 *  - Every handle owns its device memory.  Callers own the arrays they pass.
 *  - Device arrays are float64, column-major.  Vectors and dense matrices on
 *    the device are indexed in CLUSTER ORDER: position p holds the point
 *    whose original index is perm[p] (perm from h2_tree_build).
 *  - Calls enqueue work on the context's HIP stream.  Calls that choose
 *    adaptive ranks (h2_mul_intermediate, h2_recompress) synchronise that
 *    stream once per tree level to read the ranks back.
 *  - A context is not thread-safe; use one per host thread.
 *  - Arguments are validated before any launch; device failures map to
 *    H2_ERR_DEVICE.
 */
#ifndef H2_H
#define H2_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  H2_OK = 0,
  H2_ERR_ARG = 1,          /* invalid argument (NULL handle, bad size, ...) */
  H2_ERR_SHAPE = 2,        /* operands do not share the cluster trees they must share */
  H2_ERR_ALLOC = 3,        /* device or host allocation failed */
  H2_ERR_DEVICE = 4,       /* a HIP call or kernel launch failed */
  H2_ERR_NOT_REFINED = 5,  /* T^XY does not refine the target block tree T_IK */
  H2_ERR_UNSUPPORTED = 6,  /* e.g. bases of unequal rank, a block structure outside the method's */
  H2_ERR_NUMERIC = 7       /* NaN or Inf met where a finite value is required */
} h2_status;

/* Arithmetic of the bulk products (the grouped products of both phases;
 * Section 5's error control bounds what they may add).  Orthogonalisation
 * (QR), the SVDs that choose ranks and the block norms always run in
 * float64, and all stored matrices are float64.
 *   H2_FP32_BULK   operands rounded to float32, float32 accumulation (FP32
 *                  MFMA): about 1e-7 relative, accepted for eps >= 1e-6;
 *   H2_BF16X2_BULK each operand split into a bfloat16 head and a bfloat16
 *                  tail (a = a_h + a_l), products a_h b_h + a_h b_l + a_l b_h
 *                  on BF16 MFMA with float32 accumulation: about 2^-16
 *                  relative, accepted for eps >= 1e-4;
 *   H2_BF16_BULK   plain bfloat16 operands (a_h b_h only, 2^-9 rounding),
 *                  accepted for eps >= 1e-4 but not expected to meet the
 *                  2 eps bar there: offered to measure that it does not.
 * Smaller eps are H2_ERR_ARG. */
typedef enum {
  H2_FP64 = 0,         /* everything in float64 */
  H2_FP32_BULK = 1,    /* bulk products in float32 (FP32 MFMA) */
  H2_BF16X2_BULK = 2,  /* bulk products in split bfloat16 (BF16 MFMA, three products) */
  H2_BF16_BULK = 3     /* bulk products in plain bfloat16 (BF16 MFMA) */
} h2_precision;

/* Truncation rule of the rank-choosing SVDs of both phases (Section 5 error
 * control).  H2_RANK_ABS is the paper's: keep the singular values > eps of
 * the block-scaled matrix.  H2_RANK_REL_FROB is a variant: keep the fewest
 * leading singular values whose discarded tail has Frobenius norm at most
 * eps times the Frobenius norm of the whole scaled matrix (in phase 1, of its
 * part outside the kept range of V_X). */
typedef enum {
  H2_RANK_ABS = 0,
  H2_RANK_REL_FROB = 1
} h2_rank_rule;

/* Kernel functions g(x,y) of the interpolated matrices (Section 2, Example
 * "Integral operator").  Diagonal entries g(x_i, x_i) of singular kernels are 0. */
typedef enum {
  H2_K_LOG = 0,      /* log|x-y|,        diagonal 0 */
  H2_K_EXPNEG = 1,   /* exp(-|x-y|),     diagonal 1 */
  H2_K_INV4PI = 2,   /* 1/(4 pi |x-y|),  diagonal 0 (single-layer kernel, Section 7) */
  H2_K_INV = 3,      /* 1/|x-y|,         diagonal 0 */
  H2_K_DLP = 4,      /* <n(x), x-y> / (4 pi |x-y|^3), diagonal 0: the double-layer kernel of
                        Section 7, with the unit normal n(x) at the row point (needs
                        h2_compress_kernel_normals); not symmetric */
  H2_K_POLY2 = 100   /* (x.y)^2, a degree-2 polynomial reproduced exactly at order >= 3 */
} h2_kernel;

typedef struct h2_ctx h2_ctx;          /* device, stream, workspace, timers */
typedef struct h2_tree h2_tree;        /* cluster tree + block tree (standard admissibility) */
typedef struct h2_matrix h2_matrix;    /* H^2-matrix on a tree's block tree */
typedef struct h2_product h2_product;  /* phase-1 result: G on T^XY with its bases */

/* Thread-local message of the last failing call (never NULL). */
const char* h2_last_error(void);

/* Device allocator of a context: alloc returns `bytes` of device memory on
 * the context's device (aligned to at least 256 bytes) or NULL; free
 * releases such a pointer.  `user` is passed through unchanged.  The library
 * asks for large chunks (64 MiB or more), keeps them in a per-context cache
 * across calls, and hands them back to free only when the context is
 * destroyed, after every stream of the context has finished.  The callbacks
 * are called from the calling thread and, concurrently, from the library's
 * worker threads (one per auxiliary stream of the context): they must be
 * thread-safe. */
typedef void* (*h2_alloc_fn)(size_t bytes, void* user);
typedef void (*h2_free_fn)(void* p, void* user);

/* Create a context on HIP device `device` using stream `hip_stream`
 * (a hipStream_t; NULL = the default stream) and device memory from
 * alloc_fn / free_fn (both NULL: hipMalloc / hipFree; giving one of the two
 * is H2_ERR_ARG).  A NULL from alloc_fn makes the call that needed the
 * memory fail with H2_ERR_ALLOC.  device = -1 creates a host-only context
 * that accepts only h2_tree_build and the tree queries (symbolic work, no
 * device memory).  *out receives the handle.  The context also makes the
 * device's fixed scratch of h2_matvec_noalloc addressable. */
h2_status h2_ctx_create(int device, void* hip_stream, h2_alloc_fn alloc_fn, h2_free_fn free_fn, void* user,
                        h2_ctx** out);
/* Waits for the context's streams and releases the caller's hold on it.
 * Matrices and products whose device memory came from the context keep it
 * (its chunk cache, streams and allocator) until the last of them is
 * destroyed, in any order and from any thread; no new call may use the
 * context afterwards.  Handles may be destroyed at any time, also from inside
 * an allocator callback: their memory goes back to the context's cache. */
h2_status h2_ctx_destroy(h2_ctx* ctx);

/* Cluster tree (Section 2, Definition "Cluster tree") and block tree
 * (Definition "Block tree") for n points.
 *   points    host, n x dim, row-major, float64 (copied);  1 <= dim <= 3
 *   leaf_size >= 2: clusters are bisected at the median along the longest
 *             edge of their tight bounding box until every leaf holds at most
 *             leaf_size points; all leaves lie on one level.
 *   eta > 0:  standard admissibility max(diam t, diam s) <= eta dist(t, s),
 *             dist > 0; refinement stops at admissible or leaf x leaf blocks.
 *   perm_out  optional host int64[n]: perm_out[p] = original index of the
 *             point at cluster-order position p.
 * Host-only work; usable with a host-only context. */
h2_status h2_tree_build(h2_ctx* ctx, int dim, int64_t n, const double* points, int leaf_size,
                        double eta, h2_tree** out, int64_t* perm_out);

/* Sizes of a tree: out[0] = n, out[1] = dim, out[2] = depth, out[3] = #clusters,
 * out[4] = #blocks, out[5] = #admissible leaves, out[6] = #inadmissible leaves. */
h2_status h2_tree_sizes(const h2_tree* tree, int64_t out[7]);

/* Structure of a tree, host arrays sized from h2_tree_sizes (any may be NULL):
 *   cl_off, cl_size  [#clusters]  index range of each cluster in cluster order
 *                                 (clusters numbered breadth first, root 0,
 *                                 children of c are 2c+1 and 2c+2)
 *   blk_row, blk_col [#blocks]    cluster pair of each block
 *   blk_type         [#blocks]    0 = subdivided, 1 = admissible leaf, 2 = inadmissible leaf */
h2_status h2_tree_structure(const h2_tree* tree, int64_t* cl_off, int64_t* cl_size,
                            int32_t* blk_row, int32_t* blk_col, int8_t* blk_type);

/* H^2-matrix approximating the kernel matrix (g(x_i, x_j)) on tree x tree by
 * tensor Chebyshev interpolation with `order` points per axis, k = order^dim
 * (Section 2, Example "Integral operator"): leaf bases l_{t,nu}(x_i),
 * transfers l_{t,nu}(xi_{t',nu'}), couplings g(xi_t, xi_s); nearfield blocks
 * hold g(x_i, x_j).  Row and column bases coincide.  1 <= order, k <= 128. */
h2_status h2_compress_kernel(h2_ctx* ctx, const h2_tree* tree, h2_kernel kernel, int order,
                             h2_matrix** out);

/* The same with unit normals at the points (host, n x dim, row-major, in the
 * input point order of h2_tree_build; copied), for kernels that use them:
 * H2_K_DLP, the double-layer kernel <n(x), x-y>/(4 pi |x-y|^3) (Section 7).
 * With gamma(x, y) = 1/(4 pi |x-y|) that kernel is -<n(x), grad_x gamma>,
 * so gamma is interpolated in both variables and the row side is
 * differentiated: row leaf bases -<n(x_i), grad l_{t,nu}(x_i)>, column leaf
 * bases l_{s,mu}(y_j), transfers as for plain interpolation (both bases),
 * couplings gamma(xi_{t,nu}, xi_{s,mu}), nearfield entries from the kernel.
 * The interpolation boxes of this kernel are the bounding cubes of the
 * cluster boxes (a cluster on one face of a surface has a flat box, on
 * which a derivative across the face would be determined by rounding).
 * Other kernels ignore the normals.  NULL normals: H2_ERR_ARG; non-finite
 * normals: H2_ERR_NUMERIC. */
h2_status h2_compress_kernel_normals(h2_ctx* ctx, const h2_tree* tree, h2_kernel kernel, int order,
                                     const double* normals, h2_matrix** out);

/* Phase 1 for `count` independent products X[i] Y[i] (Section 4, Figure
 * "induced_basis", for the row basis and, on the adjoint pair (Y*, X*), for
 * the column basis; Section 5 block scaling; intermediate product G on
 * T^XY).  X[i] and Y[i] must be built on the same cluster tree.  A zero
 * matrix (h2_zero_like, not yet filled by h2_recompress) as a factor is
 * H2_ERR_ARG, checked before any device work: it has no bases from which
 * the induced bases could be formed, and its product is zero.
 *   eps > = 0: ranks keep the singular values > eps of the block-scaled
 *              matrices (the default rule; h2_set_rank_rule selects the
 *              relative-Frobenius variant); eps = 0 keeps every non-zero
 *              singular value and G then represents X Y exactly.
 * G_out[i] receives a new handle per product.  With count > 1 the products
 * run concurrently, up to eight at a time, each on its own streams and host
 * thread (results equal to count separate calls); HIP's default of four
 * hardware queues per process then limits their overlap, and a process
 * that batches may start with GPU_MAX_HW_QUEUES=16 (measured best).  On an
 * error every G_out[i] is left NULL. */
h2_status h2_mul_intermediate(h2_ctx* ctx, int count, const h2_matrix* const* X,
                              const h2_matrix* const* Y, double eps, h2_precision prec,
                              h2_product** G_out);

/* A zero H^2-matrix Z on `tree`'s cluster tree whose block tree, the
 * prescribed T_IK of phase 2, uses the standard admissibility condition with
 * parameter eta_Z (Section 2, Definition "Block tree"); eta_Z <= 0 takes the
 * tree's own block tree (its eta).  Phase 2 needs T^XY to refine T_IK
 * (Section 6 assumes it; H2_ERR_NOT_REFINED otherwise): a larger eta_Z gives
 * a coarser T_IK, which T^XY refines; a much smaller one may not be.
 * NaN eta_Z is H2_ERR_ARG.  Host work only (no device memory). */
h2_status h2_zero_like(h2_ctx* ctx, const h2_tree* tree, double eta_Z, h2_matrix** Z_out);

/* Phase 2 for `count` products (Section 6, Figure "basis"): builds adaptive
 * isometric nested row and column bases for Z's block tree T_IK from G and
 * stores Z <- Z + G in them.  Z[i]'s block tree must be refined by T^XY
 * (H2_ERR_NOT_REFINED otherwise).  Block-relative accuracy eps per
 * admissible block of T_IK, relative to G's block (truncation rule as set by
 * h2_set_rank_rule).
 * Z[i] may be zero (h2_zero_like) or hold a matrix on the same cluster tree
 * (a previous result, a kernel matrix, any basis ranks): Z <- Z + X Y, the
 * general operation of the paper's Introduction.  The ranges of Z's row and
 * column bases are then kept exactly (as phase 1 keeps range(V_X), Section 4
 * leaf case): the new bases start with an orthonormal basis of them
 * (numerical rank at 1e-12 relative) and add the truncated part of G outside
 * them, so the old Z is represented exactly and only G is compressed.  Z's
 * memory is replaced at the end of the call; on an error Z is unchanged.
 * The Z[i] of one call must be distinct handles (H2_ERR_ARG otherwise,
 * checked before any device work): the instances run concurrently.  The
 * G[i] are only read and may repeat. */
h2_status h2_recompress(h2_ctx* ctx, int count, h2_product* const* G, h2_matrix* const* Z,
                        double eps, h2_precision prec);

/* y <- alpha op(A) x + beta y for nvec column-major device vectors in cluster
 * order (O(nk) H^2 matrix-vector product: forward transform, couplings,
 * backward transform, nearfield).  op is 'N' or 'T'.  x and y (n x nvec
 * doubles each) must not overlap: H2_ERR_ARG, before anything is launched. */
h2_status h2_matvec(h2_ctx* ctx, const h2_matrix* A, char op, double alpha, const double* x,
                    double beta, double* y, int nvec);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as h2_matvec, through the same kernels, with every device buffer
 * beyond x and y taken from a fixed array of 64 MiB per device that the
 * library holds until the process ends (its address is resolved when a
 * context is created on the device).  Nothing is allocated: no hipMalloc,
 * hipFree, pinned-memory or event creation; descriptor tables go through the
 * context's existing pinned staging, which is reused but never grown.
 * The coefficient vectors need sum over clusters of (row rank + column rank)
 * x nvec doubles plus n x nvec for the result, each rounded up to 256 bytes;
 * with 8 MiB kept for descriptor tables this must fit in the 64 MiB, else
 * H2_ERR_ARG before anything is launched (as is a descriptor table larger
 * than the staging, before its launch and before y is written).
 * Every call on a device shares that device's array and overwrites what the
 * last call left there; calls that overlap in time on one device (several
 * contexts or host threads, different streams) race and must be serialised
 * by the caller.  Arguments and errors otherwise as h2_matvec. */
h2_status h2_matvec_noalloc(h2_ctx* ctx, const h2_matrix* A, char op, double alpha, const double* x,
                            double beta, double* y, int nvec);

/* The same for the intermediate product G. */
h2_status h2_product_matvec(h2_ctx* ctx, const h2_product* G, char op, double alpha,
                            const double* x, double beta, double* y, int nvec);

/* Dense n x n copy (cluster order) into device memory `out` with leading
 * dimension ld >= n.  For tests and measurement; O(n^2) memory. */
h2_status h2_to_dense(h2_ctx* ctx, const h2_matrix* A, double* out, int64_t ld);
h2_status h2_product_to_dense(h2_ctx* ctx, const h2_product* G, double* out, int64_t ld);

/* Expanded cluster basis matrix of cluster c (#c x rank, column-major, device
 * memory `out` with leading dimension ld >= #c) of the row (which = 0) or
 * column (which = 1) basis; for tests of projectors Q_t Q_t^*.  The basis of a
 * non-leaf cluster is expanded through the transfer matrices (eq. (transfer)). */
h2_status h2_matrix_basis(h2_ctx* ctx, const h2_matrix* A, int which, int cluster, double* out, int64_t ld);
h2_status h2_product_basis(h2_ctx* ctx, const h2_product* G, int which, int cluster, double* out, int64_t ld);

/* Ranks of a basis, host int32[#clusters]:
 *   which = 0 row basis, 1 column basis (of a matrix, or of G for products). */
h2_status h2_matrix_ranks(const h2_matrix* A, int which, int32_t* out);
h2_status h2_product_ranks(const h2_product* G, int which, int32_t* out);

/* Kinds of handles for h2_stats and h2_export. */
typedef enum { H2_HANDLE_TREE = 0, H2_HANDLE_MATRIX = 1, H2_HANDLE_PRODUCT = 2 } h2_handle_kind;

#define H2_STATS_MAX_LEVELS 32
/* Sizes and rank profile of a handle.  Block counts refer to the handle's
 * block tree (T_IJ of a tree or matrix, T^XY of a product G).  Rank fields
 * are [0] row basis, [1] column basis, per tree level from the root (levels
 * beyond H2_STATS_MAX_LEVELS - 1 are not reported); zero for trees. */
typedef struct {
  int64_t n, dim, depth, nclusters;
  int64_t nblocks, nadm, ninadm;
  int64_t triples;            /* products: terminated triples of T^XY; else 0 */
  int64_t device_bytes;       /* device memory held by the handle */
  int64_t coupling_entries;   /* stored entries of the coupling matrices */
  int64_t nearfield_entries;  /* stored entries of the nearfield blocks */
  int32_t rank_max[2];
  double rank_mean[2];
  int32_t level_rank_max[2][H2_STATS_MAX_LEVELS];
  double level_rank_mean[2][H2_STATS_MAX_LEVELS];
} h2_stats_t;

/* Fills *out for `handle` of kind h2_handle_kind.  Host data only (no device
 * work).  H2_ERR_ARG for a NULL argument or an unknown kind. */
h2_status h2_stats(const void* handle, int kind, h2_stats_t* out);

/* Writes every array of `handle` into an uncompressed NumPy .npz archive at
 * `path` (debugging and checkpoints; not timed).  Members, all 1-D unless
 * noted, in cluster order:
 *   kind; perm, cl_off, cl_size (int64, per cluster); points (n x dim,
 *   float64, cluster order); blk_row, blk_col (int32), blk_type (int8:
 *   0 subdivided, 1 admissible, 2 inadmissible) per block;
 * and for matrices and products, per basis tag in {row, col}:
 *   rank_<tag> (int32 per cluster); <tag>_leaf (float64) holding each leaf
 *   basis (#c x rank, column-major) at <tag>_leaf_off[c] .. [c + 1];
 *   <tag>_transfer holding each transfer E_c (rank c x rank parent,
 *   column-major; eq. (transfer)) at <tag>_transfer_off[c] .. [c + 1];
 *   blk_data with each block (coupling rank_row[t] x rank_col[s], or
 *   nearfield #t x #s, column-major; none for subdivided blocks) at
 *   blk_off[b] .. [b + 1].
 * Synchronises the context stream.  H2_ERR_ARG if the file cannot be
 * written or the archive would exceed 4 GiB. */
h2_status h2_export(h2_ctx* ctx, const void* handle, int kind, const char* path);

/* Sizes of a product: out[0] = #blocks of T^XY, out[1] = #admissible leaves,
 * out[2] = #inadmissible leaves, out[3] = terminated triples, out[4] = device
 * bytes held by G. */
h2_status h2_product_sizes(const h2_product* G, int64_t out[5]);

/* Step times (milliseconds) summed over the calls on this context since the
 * last read with reset != 0; out[] receives up to n entries: out[0..7]
 * device time between stream events around each step, out[8..15] host wall
 * time spent issuing it, in the order
 *   0 setup, 1 product tree and nearfield products (a third stream,
 *   overlapping steps 2/3), 2 phase-1 row, 3 phase-1 col, 4 phase-1 mat (G),
 *   5 phase-2 row, 6 phase-2 col, 7 phase-2 mat (Z).
 * The column passes run on a second stream concurrently with the row passes,
 * so steps 2/3 and 5/6 overlap in time.  The calls themselves do not wait for
 * their events; this function does (it synchronises with the streams).
 * Returns the count (0 on a NULL argument or a device error). */
int h2_step_times(h2_ctx* ctx, double* out, int n, int reset);

/* Sets the truncation rule (h2_rank_rule) of the later h2_mul_intermediate and
 * h2_recompress calls on ctx; the default is H2_RANK_ABS.  H2_ERR_ARG for an
 * unknown rule or a NULL context. */
h2_status h2_set_rank_rule(h2_ctx* ctx, int rule);

/* Level-dependent tolerances, a variant of the Section 5 error control: the
 * truncations of clusters on level l of a cluster tree of depth D use
 * eps * zeta^(D - l) in place of eps (leaves eps, each level towards the
 * root tightened by zeta), in both passes of both phases, under either rank
 * rule.  The default zeta = 1 is the paper's single tolerance.  Applies to
 * the later h2_mul_intermediate and h2_recompress calls on ctx.  H2_ERR_ARG
 * for zeta outside (0, 1] or a NULL context. */
h2_status h2_set_level_factor(h2_ctx* ctx, double zeta);

/* Memory bound of the steps that take a tree level in runs: the sums over
 * the triples of T^XY of blocks whose ranks exceed 64 (Section 3, eq. XY;
 * Section 4), the projections E_t S F_r^* and Q_t S Q_r^* of G's couplings
 * onto the blocks below them (eq. transfer), and phase 2's leaf-level C_t
 * without an old Z (Section 6, eq. ct_leaf).  Each run holds at most `bytes`
 * of device scratch (at least one block or cluster); results do not depend
 * on the bound up to rounding.  Smaller bounds lower the peak device memory
 * of a call at the cost of more, smaller launches.  bytes <= 0 restores the
 * default of 4 GiB.  Applies to the later h2_mul_intermediate and
 * h2_recompress calls on ctx.  H2_ERR_ARG for a NULL context. */
h2_status h2_set_run_scratch(h2_ctx* ctx, int64_t bytes);

/* Test hook for the error paths: the `launches`-th batched kernel launch that
 * the context's own host thread issues from now on (0 = the next one) fails
 * with H2_ERR_DEVICE before it is launched, as a host-side failure in the
 * middle of a call would; work already issued on any stream of the context
 * completes normally.  launches < 0 turns the hook off.  After the failing
 * call returns, the context and its handles remain usable.  H2_ERR_ARG for a
 * NULL context. */
h2_status h2_debug_fail_after(h2_ctx* ctx, int launches);

/* Launch timing for measurement.  h2_profile(ctx, families) makes every
 * kernel launch of a family whose bit is set in `families` (bit k for family
 * k: 0 grouped GEMM, 1 TSQR, 2 Jacobi SVD, 3 construction, 4 other;
 * H2_PROFILE_ALL sets them all, 0 turns timing off) record a pair of HIP
 * events on the context stream (a few microseconds of host time each);
 * h2_kernel_stats() resolves them (synchronising the stream) and returns,
 * for family `kind`, out[0] = total milliseconds, out[1] = launches,
 * out[2] = algorithmic flops (2mnk per product term; Householder
 * 2Nm^2 - 2m^3/3; for Jacobi, three dot products per pair and sweep
 * performed plus each rotation applied), out[3] = algorithmic bytes
 * (operands read once, outputs written once).  reset != 0 clears the counters
 * after reading.  Families whose bit is clear report zeros. */
#define H2_PROFILE_ALL 0x1F
h2_status h2_profile(h2_ctx* ctx, int families);
h2_status h2_kernel_stats(h2_ctx* ctx, int kind, double out[4], int reset);

void h2_tree_destroy(h2_tree* tree);
void h2_matrix_destroy(h2_matrix* A);
void h2_product_destroy(h2_product* G);

#ifdef __cplusplus
}
#endif
#endif /* H2_H */
