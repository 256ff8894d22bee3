// Internal declarations of the H^2 multiplication library.
//
// Host orchestration (tree.cpp, h2mat.cpp, phase1.cpp, phase2.cpp, api.cpp)
// is plain C++ over a thin device layer (dev_*) and batched kernel launchers
// (k_*).  The HIP implementations live in dev_hip.hip and kernels_*.hip.
#pragma once

#include <algorithm>
#include <chrono>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <atomic>
#include <exception>
#include <functional>
#include <mutex>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/h2.h"

namespace h2 {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  h2_status code;
  Error(h2_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};
[[noreturn]] void fail(h2_status c, const std::string& msg);
#define H2_REQUIRE(cond, code, msg) \
  do {                              \
    if (!(cond)) ::h2::fail(code, msg); \
  } while (0)

// ---------------------------------------------------------------------------
// device layer (HIP runtime; all copies are asynchronous on `stream`)
// ---------------------------------------------------------------------------
void dev_set_device(int device);
void* dev_malloc(size_t bytes);
void dev_free(void* p);
void* dev_malloc_host(size_t bytes);  // pinned, mapped, coherent
void dev_free_host(void* p);
void* dev_host_view(void* host);      // device address of pinned host memory, or nullptr
// copy from pinned host memory (its device view) with a kernel on `stream`;
// both buffers hold bytes rounded up to 256
void dev_pull(void* dst, const void* src_view, size_t bytes, void* stream);
// n ints from device memory into the device view of pinned host memory (a kernel)
void dev_push_i32(int32_t* dst_view, const int32_t* src, int n, void* stream);
void dev_h2d(void* dst, const void* src, size_t bytes, void* stream);
void dev_d2h(void* dst, const void* src, size_t bytes, void* stream);
void dev_d2d(void* dst, const void* src, size_t bytes, void* stream);
void dev_zero(void* dst, size_t bytes, void* stream);
void dev_sync(void* stream);
void* dev_stream_create();
void dev_stream_destroy(void* s);
void dev_stream_wait(void* stream, void* ev);
void* dev_event_create();
void dev_event_destroy(void* ev);
void dev_event_record(void* ev, void* stream);
float dev_event_ms(void* a, void* b);  // synchronises on b
void dev_event_sync(void* ev);

// ---------------------------------------------------------------------------
// kernel descriptors (identical layout on host and device)
// ---------------------------------------------------------------------------
// C[m x n] (ldc) = beta*C + sum_terms alpha_eff * op(A) op(B)
struct GemmOut {
  void* C;
  int64_t ldc;
  int32_t m, n;
  int32_t t0, t1;  // term range
  int32_t beta;    // 0: overwrite, 1: accumulate
  int32_t pad;
};
enum : int32_t { GT_TA = 1, GT_TB = 2, GT_BEYE = 4, GT_SCALE_MUL = 8, GT_SCALE_INV = 16 };
struct GemmTerm {
  const void* A;
  const void* B;   // unused when GT_BEYE (B = identity, k == n)
  const double* scale;  // GT_SCALE_MUL: alpha *= *scale; GT_SCALE_INV: alpha *= (*scale > 0 ? 1 / *scale : 0)
  int64_t lda, ldb;
  int32_t k, flags;
  double alpha;
};
// Chained small products C (m x n) = beta C + op(A) B op(D), all dimensions
// at most 64: op(A) is A (m x p, lda) or A^T (A stored p x m); op(D) is D^T
// (D stored n x q, ldd) or D (stored q x n); B is p x q (ldb).  One workgroup
// per item; the middle product op(A) B stays in LDS.
struct Chain3 {
  double* C;
  const double* A;
  const double* B;
  const double* D;
  int64_t ldc, lda, ldb, ldd;
  int32_t m, n, p, q;
  int32_t tA, dT, beta, pad;
};
constexpr int kChain3Max = 64;
// Grouped products driven by the product-tree triples: output o (one block of
// T^XY) = beta C + sum over the triples q in [q0, q1) whose kind equals
// F.kind of op(F.A[bx_q]) op(F.B[by_q]); the operand tables are indexed by
// the factor blocks of the triple, the inner dimension is F.k or F.ks[s_q].
struct TriOut {
  double* C;
  int64_t ldc;
  int32_t m, n;
  int32_t q0, q1;
  int32_t beta, pad;
  // block kernel only: the output is rows ro.. of op(A) times columns co.. of
  // op(B) (a 64 x 64 part of a larger output)
  int32_t ro, co;
};
struct TriFamily {
  const int32_t* tri;          // 4 ints per triple: s, bx, by, kind
  const double* const* A;      // by block of X (view)
  const int64_t* lda;
  const double* const* B;      // by block of Y (view)
  const int64_t* ldb;
  const int32_t* ks;           // inner dimension per middle cluster; null: k
  int32_t k, kind, tA, tB;
};
// R factor of the tall matrix T (N x m): T = A (transA = 0) or T = A^T where A
// is m x N column-major (transA = 1).  R (min(N,m) x m, ldr) upper, zero below.
// Householder QR (in place; reflectors below the diagonal, tau[min(m,n)]),
// R (rrows x n, upper part; zero below) copied to R if non-null.
struct QrProb {
  double* A;
  double* tau;
  double* R;
  int64_t lda, ldr;
  int32_t m, n, rrows, pad;
};
// C (m x ncols) <- Q^T C (trans = 1) or Q C (trans = 0), Q = H_0 ... H_{r-1}
struct ApplyProb {
  const double* V;
  const double* tau;
  double* C;
  int64_t ldv, ldc;
  int32_t m, nrefl, ncols, trans;
};
// R factor of T (N x m; T(i, j) = A[i + j lda], or A[j + i lda] if transA),
// restricted to the columns off..m-1, off = *col_off (nullable device int, 0
// if null): the top-left corner of R (min(N, m) x m region, zeros elsewhere)
// holds a factor F with F^T F = T'^T T', T' = T(:, off:): upper triangular
// (m - off) x (m - off) if N > m - off, else T' itself (N rows).
struct TsqrProb {
  const void* A;
  double* R;
  const int32_t* col_off;
  int64_t lda, ldr;
  int32_t N, m, transA, prec;  // prec 1: A holds float
  double* work;                 // nullable: flops of the factorization performed
};
// One-sided Jacobi SVD of R (p x m, ldr): sigma[m] (descending, zero padded),
// U (m x m, ldu, nullable) right singular vectors by descending sigma,
// rank[0] = #{sigma > max(eps, rtol * sigma_max)} (nullable).  s0 = *skip
// (nullable device int).  mode 0: R's columns < s0 are zero; all m vectors.
// mode 1: R holds the factor of the columns s0..m-1 only (as written by a
// TsqrProb with col_off = skip); vectors carry s0 leading zeros and exist for
// the nonzero singular values only (the other columns of U are zero).
struct JacobiProb {
  const double* R;
  double* U;     // may be null (values only)
  double* sigma;
  int32_t* rank;
  const int32_t* skip;
  int64_t ldr, ldu;
  int32_t p, m, mode, rule;  // rule: 0 keep sigma > max(eps, rtol sigma_max); 1 relative-Frobenius tail <= eps
  double eps, rtol;
  double* work;  // nullable: flops of the sweeps performed (dots and rotations)
};
// Spectral norm of a small matrix: out[0] = ||A||_2 for A (rows x cols,
// column-major, lda), g = min(rows, cols) <= norm2_max_dim().
struct Norm2Prob {
  const double* A;
  int64_t lda;
  int32_t rows, cols;
  double* out;
};
// block fill: A[i + j ld] = (i == j ? diag : 0) for i < rows, j < cols
struct FillItem {
  double* A;
  int64_t ld;
  int32_t rows, cols;
  double diag;
};

// launchers (descriptor arrays are device pointers)
// workgroups of the grouped products: one per output, or (work non-null,
// pairs output / first tile) one per run of kGemmTilesPerGroup tiles
constexpr int kGemmTilesPerGroup = 16;
void k_gemm_sum(const GemmOut* outs, const GemmTerm* terms, const int32_t* work, int ngroups, int prec,
                void* stream);
// prec 1: the products run on FP32 MFMA (operands rounded to FP32, FP32
// accumulation, FP64 storage); 0: FP64 MFMA
void k_gemm_tri(const TriOut* outs, const int32_t* tiles, int ntiles, const TriFamily& fam, int prec, void* stream);
// one workgroup per output of at most 64 x 64 (untransposed operands)
void k_gemm_tri_block(const TriOut* outs, int nouts, const TriFamily& fam, int prec, void* stream);
void k_chain3(const Chain3* items, int n, void* stream);
// The coefficients S_b of the admissible part of G on one level of T^XY,
// one workgroup per block b = b0 + i (Section 6 opening with reading R14):
//   TAA = sum over the block's AA triples of S_X P S_Y          (k x k)
//   TNA = sum over NA triples of A_{t,s} S_Y                     (kt x k)
//   MAN = sum over AN triples of S_X A^c_{r,s}^*                 (k x kr)
//   S_b = TNA R^c_r^* + R_t (TAA R^c_r^* + MAN)                  (kt x kr)
// with R_t = [R_{X,t}; 0] (row pass) and R^c_r (column pass).  Every
// dimension at most 64.
struct GformArgs {
  // whole T^XY and the blocks of X and Y
  const int32_t* bt;        // row cluster of block b at bt[2b], column cluster at bt[2b + 1]
  const int32_t* tri_ptr;   // triples of block b: [tri_ptr[b], tri_ptr[b + 1])
  const int32_t* tri;       // 4 ints per triple: s, bx, by, kind
  const double* const* SX;  // per block of X (couplings where admissible)
  const int64_t* ldSX;
  const double* const* SY;  // per block of Y
  const int64_t* ldSY;
  const double* const* PS;  // per block of Y: P_{XY,s} S_{Y,sr} (k x k, ld k), admissible blocks
  // the level's own (every factor of a triple of a block on level l lies on level l)
  const double* const* Ar;  // per block bx0 + i of X: A_{t,s} (kt x k), non-admissible blocks
  const int64_t* ldAr;
  const double* const* Ac;  // per block by0 + i of Y: A^c (kr x k), non-admissible blocks
  const int64_t* ldAc;
  const int32_t* krow;      // per cluster c0 + i: rank of the row basis
  const int32_t* kcol;      // per cluster c0 + i: rank of the column basis
  const double* const* Rr;  // per cluster: [R_{X,t}; 0] (krow x k, ld max(krow, 1))
  const double* const* Rc;  // per cluster: [R^c_{Y,r}; 0] (kcol x k, ld max(kcol, 1))
  double* const* S;         // per block b0 + i of T^XY: S_b (kt x kr, ld max(kt, 1))
  int32_t b0, c0, bx0, by0, k, ktmax, krmax;
};
// dynamic LDS in doubles of a launch (k, the level's largest kt and kr)
size_t gform_lds_doubles(int k, int ktmax, int krmax);
void k_gform(const GformArgs& a, int nblocks, int prec, void* stream);
// Factorization launches: lds_doubles is the dynamic LDS of the launch (a
// problem whose working set fits it runs in LDS), slot the doubles of global
// scratch per workgroup for the others (0: none); scratch then holds
// slot * min(n, 1024) doubles.  lds_limit_doubles() is the device maximum.
// TSQR sizes its row chunks from the device maximum: a problem runs in LDS
// iff tsqr_lds_need(m, limit) > 0, and lds_doubles must cover that need.
int lds_limit_doubles();
size_t qr_need_doubles(int m, int n);
size_t tsqr_lds_need(int m, int cap);
size_t tsqr_scratch_need(int m);
size_t tsqr_chunk_need(int m, int cap);  // LDS doubles of the chunks-only mode
// register-blocked TSQR variants (1..3; 0 = none fits) for problems whose
// factored width is at most m, and their LDS need in doubles
int tsqr_rb_variant(int m, int cap);
size_t tsqr_rb_need(int variant, int m);
int tsqr_rb_chunk(int variant);  // rows factored per step sequence
void k_tsqr_rb(int variant, const TsqrProb* probs, int n, size_t lds_doubles, void* stream);
size_t jacobi_need_doubles(int p, int m, int mode);
void k_qr(const QrProb* probs, int n, int lds_doubles, void* stream);
void k_apply(const ApplyProb* probs, const int32_t* work, int nwork, int lds_doubles, void* stream);
void k_tsqr(const TsqrProb* probs, int n, size_t lds_doubles, size_t slot, double* scratch, void* stream);
// problems with m <= jacobi_small_max_m(): one wavefront each, per_doubles of
// LDS each (4 per workgroup)
int jacobi_small_max_m();
int jacobi_max_len();
void k_jacobi_small(const JacobiProb* probs, int n, int per_doubles, void* stream);
// replaces the rank written by a Jacobi launch with the relative-Frobenius
// rank of the singular values it wrote (problems with rule 1)
void k_rank_relf(const JacobiProb* probs, int n, void* stream);
// spectral norms: one wavefront per problem, per_doubles = norm2_need_doubles
// of the largest g of the launch and the staging chunk (16, 32 or 64 samples)
int norm2_max_dim();
size_t norm2_need_doubles(int g, int chunk);
void k_norm2(const Norm2Prob* probs, int n, int per_doubles, int chunk, void* stream);
// medium problems (m <= jacobi_mid_max_m()) take 256-thread workgroups,
// larger ones 1024 (wide)
int jacobi_mid_max_m();
void k_jacobi(const JacobiProb* probs, int n, int lds_doubles, size_t slot, double* scratch, bool wide,
              void* stream);
void k_fill(const FillItem* items, int n, void* stream);
// groups g of values *vals[i], i in [gptr[g], gptr[g+1]): values at most
// rtol times the group's largest become 0
void k_drop_small(double* const* vals, const int32_t* gptr, int ngroups, double rtol, void* stream);

// interpolation / kernel evaluation
struct ChebLeaf {   // V[i, nu] for leaf cluster c
  double* V;
  int64_t ldv, off;  // point offset in cluster order
  int32_t c, size;
};
struct ChebPair {   // transfer E_c (c, parent) or coupling S_ts (t, s)
  double* out;
  int64_t ld;
  int32_t a, b;
};
struct NearBlock {
  double* out;
  int64_t ld, off_t, off_s;
  int32_t size_t_, size_s, diag, pad;
};
void k_cheb_leaf(const ChebLeaf* d, int n, const double* pts, const double* lo, const double* hi,
                 int dim, int order, void* stream);
void k_cheb_transfer(const ChebPair* d, int n, const double* lo, const double* hi, int dim,
                     int order, void* stream);
void k_cheb_coupling(const ChebPair* d, int n, const double* lo, const double* hi, int dim,
                     int order, int kernel, void* stream);
// leaves of the double-layer row basis: -<n(x_i), grad l_{c,nu}(x_i)>
void k_cheb_leaf_dn(const ChebLeaf* d, int n, const double* pts, const double* nrm, const double* lo,
                    const double* hi, int dim, int order, void* stream);
// nrm: unit normals at the points (cluster order), read for H2_K_DLP only
void k_nearfield(const NearBlock* d, int n, const double* pts, const double* nrm, int dim, int kernel,
                 void* stream);

// segmented sums of squares: out[i] = sum over items of segment i of ||M||_F^2
struct SumsqItem {
  const double* M;
  int64_t ld;
  int32_t rows, cols;
};
void k_sumsq(const SumsqItem* items, const int32_t* seg_ptr, int nseg, double* out, int mode,
             void* stream);  // mode 1: out = s > 0 ? 1/sqrt(s) : 0
// y (rows x cols, ldy) <- alpha x + beta y (beta = 0 ignores y)
void k_axpby(int64_t rows, int64_t cols, double alpha, const double* x, int64_t ldx, double beta,
             double* y, int64_t ldy, void* stream);

// ---------------------------------------------------------------------------
// host structures
// ---------------------------------------------------------------------------
struct TreeH {  // complete binary cluster tree of uniform depth, breadth-first ids
  int dim = 0, depth = 0, ncl = 0;
  int64_t n = 0;
  std::vector<int64_t> off, size, perm;
  std::vector<double> pts;      // permuted points, n x dim row-major
  std::vector<double> lo, hi;   // interpolation boxes (widened), ncl x dim
  std::vector<double> blo, bhi; // tight boxes, ncl x dim
  static int level(int c) {
    int l = 0;
    while ((2 << l) - 1 <= c) ++l;
    return l;
  }
  static int first(int l) { return (1 << l) - 1; }
  static int parent(int c) { return (c - 1) / 2; }
  bool leaf(int c) const { return level(c) == depth; }
  bool same_as(const TreeH& o) const { return n == o.n && depth == o.depth && perm == o.perm; }
};

enum : int8_t { BT_SPLIT = 0, BT_ADM = 1, BT_INADM = 2 };
struct BlockTreeH {  // level-aligned block tree; children of a split block are 4 consecutive ids
  std::vector<int32_t> t, s, child0;
  std::vector<int8_t> type;
  std::vector<int32_t> lvl;        // blocks of level l: [lvl[l], lvl[l+1])
  std::vector<int32_t> row_ptr, row_blk, col_ptr, col_blk;  // CSR by row / column cluster
  int64_t n_adm = 0, n_inadm = 0;
  int nblocks() const { return (int)t.size(); }
  void finalize(int ncl);          // builds CSRs (sorted by the other cluster)
  int find(int tt, int ss) const;  // block id or -1
};

struct h2_tree_impl;

// nested cluster basis on the device
struct Basis {
  std::vector<int32_t> rank;
  std::vector<double*> leaf;      // leaf c: #c x rank[c]
  std::vector<int64_t> leaf_ld;
  std::vector<double*> tr;        // non-root c: rank[c] x rank[parent]
  std::vector<int64_t> tr_ld;
  void resize(int ncl) {
    rank.assign(ncl, 0);
    leaf.assign(ncl, nullptr);
    leaf_ld.assign(ncl, 1);
    tr.assign(ncl, nullptr);
    tr_ld.assign(ncl, 1);
  }
};

struct H2Core {
  std::shared_ptr<TreeH> ct;
  std::shared_ptr<BlockTreeH> bt;
  Basis V, W;
  std::vector<double*> blk;  // coupling rank_V[t] x rank_W[s] (ld rank_V[t]) or nearfield #t x #s (ld #t)
  int64_t ld_of(int b) const {
    return bt->type[b] == BT_ADM ? (int64_t)std::max(1, V.rank[bt->t[b]]) : ct->size[bt->t[b]];
  }
};

}  // namespace h2

// ---------------------------------------------------------------------------
// context and arenas
// ---------------------------------------------------------------------------
struct h2_ctx;

namespace h2 {

// tolerance of the truncations on level l of a tree of depth D (the
// level-dependent variant; zeta = 1 gives eps on every level)
inline double level_eps(const h2_ctx* ctx, double eps, int D, int l);

struct Arena {
  h2_ctx* ctx = nullptr;
  h2_ctx* owner = nullptr;  // root context referenced by a handle's arena (bind)
  std::vector<std::pair<char*, size_t>> chunks;
  size_t cur = 0, used = 0, total = 0;
  // fixed region (device scratch of the entry point that allocates nothing):
  // when set, alloc() bumps inside it and fails once it is exhausted
  char* fixed = nullptr;
  size_t fixed_cap = 0, fixed_used = 0;
  void* alloc(size_t bytes);
  template <class T>
  T* get(size_t count) { return (T*)alloc(count * sizeof(T)); }
  void reset() { cur = 0; used = 0; }
  // the arena of a handle: memory from c, whose root context stays alive
  // (h2_ctx_destroy is deferred) until the arena is gone
  void bind(h2_ctx* c);
  void release();  // chunks go back to the context (its returned list)
  void swap(Arena& o) {
    std::swap(ctx, o.ctx);
    std::swap(owner, o.owner);
    chunks.swap(o.chunks);
    std::swap(cur, o.cur);
    std::swap(used, o.used);
    std::swap(total, o.total);
    std::swap(fixed, o.fixed);
    std::swap(fixed_cap, o.fixed_cap);
    std::swap(fixed_used, o.fixed_used);
  }
  ~Arena();
};

// Scratch of one scope on one context: allocated like the workspace, its
// chunks go back to that context's cache when the scope ends (or at
// reset()), where only the same context takes them again, after the work
// already queued on its stream.  Per-level temporaries live here, so that a
// pass holds one level's scratch at a time rather than the sum over levels.
struct ScopedArena : Arena {
  explicit ScopedArena(h2_ctx* c) { ctx = c; }
  ScopedArena(const ScopedArena&) = delete;
  ScopedArena& operator=(const ScopedArena&) = delete;
};

}  // namespace h2

namespace h2 {
enum KernelKind { KK_GEMM = 0, KK_TSQR = 1, KK_JACOBI = 2, KK_BUILD = 3, KK_OTHER = 4, KK_COUNT = 5 };
struct KernelStat {
  double ms = 0, flops = 0, bytes = 0;
  int64_t launches = 0;
};
struct PendingLaunch {
  void* a;
  void* b;
  int kind;
  double flops, bytes;
  const double* work = nullptr;  // pinned host copy of per-problem flops (replaces flops)
  int nwork = 0;
};
}  // namespace h2

constexpr size_t kRunScratchDefault = (size_t)4 << 30;

struct h2_ctx {
  int device = -1;
  void* stream = nullptr;
  bool host_only = true;
  h2::Arena ws;                        // per-call workspace
  std::vector<std::pair<char*, size_t>> cache;  // free device chunks (touched by the context's own thread)
  // chunks handed back by destroyed handles, from any thread (also from
  // inside an allocator callback): merged into `cache` before it is searched
  std::mutex ret_mu;
  std::vector<std::pair<char*, size_t>> returned;
  // root contexts: idle chunks of every context of the family (the root,
  // its auxiliary chain and its lanes), pooled at the start of each call
  // once the previous call's work is ordered before the root stream; any
  // context of the family takes from it, and it is handed back to the
  // allocator when an allocation fails
  std::mutex pool_mu;
  std::vector<std::pair<char*, size_t>> pool;
  h2_ctx* root = nullptr;              // auxiliary contexts: the context they belong to
  // references on a root context: the caller's (dropped by h2_ctx_destroy)
  // plus one per handle arena holding its memory; the last drop deletes it
  std::atomic<int> refs{1};
  char* stage = nullptr;               // pinned staging for descriptor uploads
  char* stage_dev = nullptr;           // its device view (nullptr: runtime copies)
  size_t stage_cap = 0, stage_used = 0;
  std::vector<void*> events;
  std::vector<int> ev_step;            // step id of each recorded event interval
  double step_ms[8] = {0};
  double host_ms[8] = {0};             // host wall time between step_begin and step_end
  std::chrono::steady_clock::time_point host_t0[8];
  int prec = 0;                        // bulk precision of the running call
  int rank_rule = 0;                   // h2_rank_rule of the truncating SVDs
  double level_factor = 1.0;           // zeta: level l truncates at eps zeta^(depth - l)
  // bound on the device scratch of one run of blocks or clusters in the
  // steps that take a level in runs (h2_set_run_scratch)
  size_t run_scratch = kRunScratchDefault;
  int profile = 0;                     // bit k: time the launches of kernel family k
  int fail_after = -1;                 // test hook: launches left before an injected failure (-1: off)
  h2_alloc_fn alloc_fn = nullptr;      // caller's device allocator (nullptr: hipMalloc / hipFree)
  h2_free_fn free_fn = nullptr;
  void* alloc_user = nullptr;
  char* scratch_dev = nullptr;         // device address of the fixed scratch on this device
  bool no_alloc = false;               // inside an entry point that allocates nothing
  std::vector<void*> ev_pool;          // reusable events for launch timing
  std::vector<std::pair<double*, size_t>> prof_host;  // pinned chunks for per-problem work counts
  size_t prof_chunk = 0, prof_used = 0;
  std::vector<h2::PendingLaunch> pending;
  h2::KernelStat kstat[h2::KK_COUNT];
  // second context on the same device (own stream, workspace, staging) for
  // the column passes, which run concurrently with the row passes
  h2_ctx* aux = nullptr;
  // root contexts: one context per concurrent instance of a batched call
  // (each with its own auxiliary chain), created on first use
  std::vector<h2_ctx*> lanes;
  void* drain = nullptr;  // auxiliary contexts: end of the last run's work on the stream
  bool own_stream = false;
  ~h2_ctx();
};

namespace h2 {
inline double level_eps(const h2_ctx* ctx, double eps, int D, int l) {
  double e = eps;
  for (int j = l; j < D; ++j) e *= ctx->level_factor;
  return e;
}
}  // namespace h2

struct h2_tree {
  std::shared_ptr<h2::TreeH> ct;
  std::shared_ptr<h2::BlockTreeH> bt;
  double eta = 0;
};

struct h2_matrix {
  h2_ctx* ctx = nullptr;
  h2::H2Core c;
  h2::Arena mem;
  h2::Arena mem_aux;  // results of the column pass (allocated by the auxiliary context)
  bool zero = false;
};

struct h2_product {
  h2_ctx* ctx = nullptr;
  h2::H2Core c;
  h2::Arena mem;
  h2::Arena mem_aux;  // results of the column pass (allocated by the auxiliary context)
  h2::Arena mem_nf;   // dense leaf blocks (allocated by the second auxiliary context)
  int64_t n_triples = 0;
};

namespace h2 {

// uploads (pinned staging -> workspace), sync helper resets the staging.
// stage_alloc hands out pinned host space (it may wait for earlier copies),
// stage_upload enqueues its copy into fresh workspace.
char* stage_alloc(h2_ctx* ctx, size_t bytes);
void* stage_upload(h2_ctx* ctx, const char* h, size_t bytes);
void* upload_bytes(h2_ctx* ctx, const void* src, size_t bytes);
template <class T, class A>
T* upload(h2_ctx* ctx, const std::vector<T, A>& v) {
  if (v.empty()) return nullptr;
  return (T*)upload_bytes(ctx, v.data(), v.size() * sizeof(T));
}
// the same for a table read only by the launch issued next (small tables are
// read from the staging itself; see stage_launch)
void* stage_launch(h2_ctx* ctx, const char* h, size_t bytes);
void* upload_launch_bytes(h2_ctx* ctx, const void* src, size_t bytes);
template <class T>
T* upload_launch(h2_ctx* ctx, const std::vector<T>& v) {
  if (v.empty()) return nullptr;
  return (T*)upload_launch_bytes(ctx, v.data(), v.size() * sizeof(T));
}
// asynchronous copy of n device ints into pinned staging; the host pointer
// holds them after the next ctx_sync and until the next staging allocation
const int32_t* read_back(h2_ctx* ctx, const int32_t* dev, int n);
void ctx_sync(h2_ctx* ctx);

// launch timing (when bit `kind` of ctx->profile is set): events around one launch
struct LaunchTimer {
  h2_ctx* ctx;
  void* a = nullptr;
  int kind;
  double flops, bytes;
  const double* work = nullptr;
  int nwork = 0;
  LaunchTimer(h2_ctx* c, int k, double f, double b);
  ~LaunchTimer();
};
// profiling only: device array of n per-problem work counts, and the pinned
// host array its values are copied to once the launch is done
struct WorkCounts {
  double* dev = nullptr;
  double* host = nullptr;
  int n = 0;
};
WorkCounts work_counts(h2_ctx* ctx, int n, int kind);
void kernel_stats_collect(h2_ctx* ctx);

// step timing with stream events
void step_begin(h2_ctx* ctx, int step);
void step_end(h2_ctx* ctx, int step);
void steps_collect(h2_ctx* ctx);

void* pool_event(h2_ctx* ctx);
// the auxiliary context of ctx (created on first use); the auxiliary
// context's own one, aux_ctx(aux_ctx(ctx)), is a third stream
h2_ctx* aux_ctx(h2_ctx* ctx);
// instances of a batched call run concurrently, at most this many at a time,
// each on a lane context of the root context (own stream, workspace and
// staging, and its own auxiliary contexts for its column pass and dense
// products); lane_ctx(ctx, w) creates lane w on first use
constexpr int kBatchLanes = 8;
h2_ctx* lane_ctx(h2_ctx* ctx, int w);
// Runs f(aux) on a host thread, on the auxiliary stream, ordered after the
// work queued so far on ctx->stream.  join() waits for the thread, makes
// ctx->stream wait for the auxiliary work, and rethrows its exception.
struct AuxRun {
  h2_ctx* ctx;
  h2_ctx* aux;
  std::thread th;
  std::exception_ptr err;
  bool joined = false;
  AuxRun(h2_ctx* c, std::function<void(h2_ctx*)> f);
  AuxRun(h2_ctx* c, h2_ctx* a, std::function<void(h2_ctx*)> f);  // on a given auxiliary context
  void join();
  ~AuxRun();
};
// step times and launch statistics of the auxiliary context, folded into ctx
void aux_collect(h2_ctx* ctx);

// batched launch builders
struct GemmBatch {
  std::vector<GemmOut> outs;
  std::vector<GemmTerm> terms;
  int prec = 0;
  // starts a new output; subsequent term() calls accumulate into it
  void out(double* C, int64_t ldc, int m, int n, bool accumulate = false);
  void term(const double* A, int64_t lda, bool tA, const double* B, int64_t ldb, bool tB, int k,
            double alpha = 1.0, const double* scale = nullptr, int scale_mode = 0);
  void copy(const double* A, int64_t lda, bool tA, int k, double alpha = 1.0,
            const double* scale = nullptr, int scale_mode = 0);  // op(A) * I_k
  void run(h2_ctx* ctx);
  bool empty() const { return outs.empty(); }
};
// chained products C = beta C + op(A) B op(D) (one launch)
struct Chain3Batch {
  std::vector<Chain3> items;
  // false when a dimension exceeds kChain3Max (the caller then uses GemmBatch)
  static bool fits(int m, int n, int p, int q) {
    return m <= kChain3Max && n <= kChain3Max && p <= kChain3Max && q <= kChain3Max;
  }
  void add(double* C, int64_t ldc, int m, int n, const double* A, int64_t lda, bool tA, int p,
           const double* B, int64_t ldb, int q, const double* D, int64_t ldd, bool dT, bool accumulate);
  void run(h2_ctx* ctx);
};
// outputs of one triple family (one launch)
struct TriBatch {
  std::vector<TriOut> outs;
  TriFamily fam{};
  // untransposed operands: one workgroup per output of at most 64 x 64; out()
  // then cuts a larger output into 64 x 64 parts
  bool block = false;
  int prec = 0;
  void out(double* C, int64_t ldc, int m, int n, int q0, int q1, bool accumulate = false);
  void run(h2_ctx* ctx, double flops);
};
struct QrBatch {
  std::vector<QrProb> p;
  void add(double* A, int64_t lda, int m, int n, double* tau, double* R, int64_t ldr, int rrows);
  void run(h2_ctx* ctx);
};
struct ApplyBatch {
  std::vector<ApplyProb> p;
  void add(const double* V, int64_t ldv, const double* tau, int m, int nrefl, double* C,
           int64_t ldc, int ncols, bool trans);
  void run(h2_ctx* ctx);
};
struct FillBatch {
  std::vector<FillItem> items;
  void add(double* A, int64_t ld, int rows, int cols, double diag = 0.0) {
    if (rows > 0 && cols > 0) items.push_back({A, std::max<int64_t>(ld, 1), rows, cols, diag});
  }
  void run(h2_ctx* ctx);
};
struct TsqrBatch {
  std::vector<TsqrProb> p;
  int max_m = 0;
  void add(const void* A, int64_t lda, int N, int m, bool transA, double* R, int64_t ldr,
           int prec = 0, const int32_t* col_off = nullptr);
  void run(h2_ctx* ctx);
};
struct JacobiBatch {
  std::vector<JacobiProb> p;
  int max_m = 0;
  void add(const double* R, int64_t ldr, int p_, int m, double* U, int64_t ldu, double* sigma,
           int32_t* rank, double eps, double rtol = 0.0, const int32_t* skip = nullptr, int mode = 1,
           int rule = 0);
  void run(h2_ctx* ctx);
};
// sigma_max of many small matrices: tsqr + jacobi (values only); sig[i] = sigma_max
struct NormBatch {
  struct Item {
    const double* A;  // stored rows x cols, column-major
    int64_t lda;
    int rows, cols;
  };
  std::vector<Item> items;
  // drop rule of the Section 5 scaling: sigma_max of an item at most
  // drop_rtol times the largest of its group is set to 0 (the block is then
  // dropped); group[i] numbers the groups from 0 in item order (empty: off)
  double drop_rtol = 0.0;
  std::vector<int32_t> group;
  void add(const double* A, int64_t lda, int rows, int cols, int grp = -1) {
    items.push_back({A, lda, rows, cols});
    if (grp >= 0) group.push_back(grp);
  }
  std::vector<const double*> run(h2_ctx* ctx);  // device pointer to sigma_max of each item
};
// a block whose spectral norm is at most this fraction of the largest block
// norm of its level (same pass and kind) is zero up to rounding
constexpr double kBlockRtol = 1e-12;

// drops a reference on a root context; the last one deletes it
void ctx_unref(h2_ctx* root);
// start of a call on a root context (the previous call's work is ordered
// before its stream): every context of the family rewinds its workspace and
// hands its idle chunks to the root's pool
void pool_idle_memory(h2_ctx* root);
// start of one instance of a batched call on ctx: ctx and its auxiliary
// chain rewind their workspaces (the previous instance's work on them is
// ordered before ctx's stream)
void rewind_workspaces(h2_ctx* ctx);

// device memory of a context: the caller's allocator callbacks when given,
// else the HIP runtime
void* ctx_malloc(h2_ctx* ctx, size_t bytes);
void ctx_free(h2_ctx* ctx, void* p);

// zeroed device buffer from an arena
double* zeros(h2_ctx* ctx, Arena& a, size_t count);

// trees
std::shared_ptr<TreeH> build_cluster_tree(int dim, int64_t n, const double* pts, int leaf_size);
std::shared_ptr<BlockTreeH> build_block_tree(const TreeH& rt, const TreeH& ct, double eta);

// product block tree with triples
enum : int8_t { TK_AA = 0, TK_AN = 1, TK_NA = 2, TK_NN = 3, TK_SPLIT = 4 };
struct Triple {
  int32_t s, bx, by;  // middle cluster, block of X (view coords), block of Y
  int32_t kind;       // laid out as the 4 ints a TriFamily reads
};
// allocator whose resize leaves plain data uninitialised (large host tables
// written in parallel right after they are sized: their pages are first
// touched by the threads that fill them)
template <class T>
struct DefaultInit : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = DefaultInit<U>;
  };
  using std::allocator<T>::allocator;
  template <class U>
  void construct(U* p) noexcept {
    ::new ((void*)p) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new ((void*)p) U(std::forward<A>(a)...);
  }
};
struct ProductTreeH {
  std::shared_ptr<BlockTreeH> bt;           // T^XY
  std::vector<int32_t> tri_ptr;             // per block
  std::vector<Triple, DefaultInit<Triple>> tri;
  std::vector<int32_t> kind_cnt;            // 4 per block: triples of each kind
  int64_t n_terminated = 0;
};

// views of an H^2-matrix or its adjoint
struct View {
  const H2Core* m = nullptr;
  bool T = false;
  const Basis& rowb() const { return T ? m->W : m->V; }
  const Basis& colb() const { return T ? m->V : m->W; }
  const BlockTreeH& bt() const { return *m->bt; }
  // block ids whose view-row is t (sorted by view-column)
  void row_blocks(int t, const int32_t*& b, int& cnt) const {
    const auto& B = *m->bt;
    if (!T) {
      b = B.row_blk.data() + B.row_ptr[t];
      cnt = B.row_ptr[t + 1] - B.row_ptr[t];
    } else {
      b = B.col_blk.data() + B.col_ptr[t];
      cnt = B.col_ptr[t + 1] - B.col_ptr[t];
    }
  }
  int vrow(int b) const { return T ? m->bt->s[b] : m->bt->t[b]; }
  int vcol(int b) const { return T ? m->bt->t[b] : m->bt->s[b]; }
  int find(int t, int s) const { return T ? m->bt->find(s, t) : m->bt->find(t, s); }
  int8_t type(int b) const { return m->bt->type[b]; }
  const double* ptr(int b) const { return m->blk[b]; }
  int64_t ld(int b) const { return m->ld_of(b); }
};
ProductTreeH build_product_tree(const View& X, const View& Y, int ncl);

// matrices
// normals: host n x dim in the input point order (H2_K_DLP only; else null)
void compress_kernel(h2_ctx* ctx, const h2_tree* tree, int kernel, int order, const double* normals,
                     h2_matrix* out);
void zero_like(h2_ctx* ctx, const h2_tree* tree, double eta_Z, h2_matrix* out);
void matvec(h2_ctx* ctx, const H2Core& A, bool trans, double alpha, const double* x, double beta,
            double* y, int nvec);
void to_dense(h2_ctx* ctx, const H2Core& A, double* out, int64_t ld);
void basis_dense(h2_ctx* ctx, const H2Core& A, int which, int cluster, double* out, int64_t ld);

// the entry point that allocates nothing: a fixed device array of this size
// per device (coefficient vectors, result staging and large descriptor
// tables of one call); kNoAllocTableReserve of it is kept for the tables
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr size_t kNoAllocTableReserve = (size_t)8 << 20;
char* noalloc_scratch_resolve(int device);
void matvec_noalloc(h2_ctx* ctx, const H2Core& A, bool trans, double alpha, const double* x, double beta,
                    double* y, int nvec);

// Bases keeping range(K) exactly plus the truncated SVD of the rest of C
// (Section 4, leaf case): K (m x kc, ldk), C (m x nc, ldc; overwritten).
struct KeptItem {
  int m;
  const double* K;
  int64_t ldk;
  int kc;
  double* C;
  int64_t ldc;
  int nc;
};
struct KeptOut {
  std::vector<int32_t> k1, k2;  // numerical rank of K; kept singular values of the rest
  std::vector<double*> Q;       // m x (k1 + k2), ld m (from `keep`)
  std::vector<double*> RKP;     // Q^* K = [R_K; 0]: (k1 + k2) x kc, ld max(k1 + k2, 1) (workspace)
};
// one launch per step over all items; reads the ranks back (one stream sync)
void kept_compress(h2_ctx* ctx, const std::vector<KeptItem>& items, double eps, Arena& keep, KeptOut& out);

// h2_stats / h2_export
void handle_stats(const void* handle, int kind, h2_stats_t* out);
void export_handle(h2_ctx* ctx, const void* handle, int kind, const std::string& path);

// phases
void phase1(h2_ctx* ctx, const h2_matrix* X, const h2_matrix* Y, double eps, int prec,
            h2_product* G);
void phase2(h2_ctx* ctx, h2_product* G, h2_matrix* Z, double eps, int prec);

}  // namespace h2
