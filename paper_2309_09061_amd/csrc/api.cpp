// extern "C" entry points of include/h2.h.  Arguments are validated here
// before any launch; internal errors are exceptions mapped to status codes.
#include <algorithm>
#include <cmath>
#include <string>

#include "internal.h"

using namespace h2;

static thread_local std::string g_err = "no error";

template <class F>
static h2_status guard(F&& f) {
  try {
    f();
    return H2_OK;
  } catch (const Error& e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return H2_ERR_ALLOC;
  } catch (const std::exception& e) {
    g_err = e.what();
    return H2_ERR_DEVICE;
  }
}

static void need_device(const h2_ctx* ctx) {
  H2_REQUIRE(ctx, H2_ERR_ARG, "NULL context");
  H2_REQUIRE(!ctx->host_only, H2_ERR_ARG, "host-only context: no device work possible");
  dev_set_device(ctx->device);
}

// Smallest eps of each bulk precision: FP32 rounding (about 6e-8 relative,
// with growth over the levels) stays within the 2 eps bar only above 1e-6,
// the split bfloat16 products (about 2^-16 = 1.5e-5 relative) above 1e-4
static void check_precision(int prec, double eps) {
  H2_REQUIRE(prec >= H2_FP64 && prec <= H2_BF16_BULK, H2_ERR_ARG, "unknown precision");
  H2_REQUIRE(prec != H2_FP32_BULK || eps >= 1e-6, H2_ERR_ARG,
             "FP32 bulk products need eps >= 1e-6 (FP32 rounding would exceed 2 eps)");
  H2_REQUIRE(prec < H2_BF16X2_BULK || eps >= 1e-4, H2_ERR_ARG,
             "bfloat16 bulk products need eps >= 1e-4 (their rounding would exceed 2 eps)");
}

// The workspace of the previous call is reused at once: every later launch
// is ordered after the earlier ones on the context stream, and the auxiliary
// stream's work of a call is ordered after the context stream's work queued
// before it.
static void begin_call(h2_ctx* ctx) { pool_idle_memory(ctx); }

// Runs body(lane, i) for the instances i = 0..count-1 of a batched call, at
// most kBatchLanes at a time, each lane on its own host thread, stream and
// workspace; instances are taken largest first (weight w[i]) from a shared
// counter.  Every lane is ordered after the work queued on ctx->stream so
// far, and ctx->stream after every lane's work.  The first exception stops
// the lanes from taking further instances and is rethrown once all have
// been joined.
static void run_lanes(h2_ctx* ctx, int count, const std::vector<int64_t>& w,
                      const std::function<void(h2_ctx*, int)>& body) {
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return w[a] > w[b]; });
  const int nl = std::min(count, h2::kBatchLanes);
  std::atomic<int> next{0};
  std::atomic<bool> stop{false};
  std::vector<std::unique_ptr<h2::AuxRun>> runs;
  std::exception_ptr first;
  try {
    for (int l = 0; l < nl; ++l)
      runs.push_back(std::make_unique<h2::AuxRun>(ctx, h2::lane_ctx(ctx, l), [&](h2_ctx* a) {
        for (;;) {
          const int j = next.fetch_add(1);
          if (j >= count || stop.load()) return;
          try {
            body(a, order[j]);
          } catch (...) {
            stop.store(true);
            throw;
          }
        }
      }));
  } catch (...) {
    stop.store(true);
    first = std::current_exception();
  }
  for (auto& r : runs) {
    try {
      r->join();
    } catch (...) {
      if (!first) first = std::current_exception();
    }
  }
  if (first) std::rethrow_exception(first);
}

extern "C" {

const char* h2_last_error(void) { return g_err.c_str(); }

h2_status h2_ctx_create(int device, void* hip_stream, h2_alloc_fn alloc_fn, h2_free_fn free_fn, void* user,
                        h2_ctx** out) {
  return guard([&] {
    H2_REQUIRE(out, H2_ERR_ARG, "NULL output");
    *out = nullptr;
    H2_REQUIRE(device >= -1, H2_ERR_ARG, "bad device");
    H2_REQUIRE((alloc_fn == nullptr) == (free_fn == nullptr), H2_ERR_ARG,
               "give both allocator callbacks or neither");
    auto* c = new h2_ctx();
    c->device = device;
    c->stream = hip_stream;
    c->host_only = device < 0;
    c->ws.ctx = c;
    c->alloc_fn = alloc_fn;
    c->free_fn = free_fn;
    c->alloc_user = user;
    if (!c->host_only) {
      try {
        dev_set_device(device);
        c->stage_cap = (size_t)16 << 20;
        c->stage = (char*)dev_malloc_host(c->stage_cap);
        c->stage_dev = (char*)dev_host_view(c->stage);
        c->scratch_dev = noalloc_scratch_resolve(device);
      } catch (...) {
        delete c;
        throw;
      }
    }
    *out = c;
  });
}

h2_status h2_ctx_destroy(h2_ctx* ctx) {
  return guard([&] {
    if (!ctx) return;
    H2_REQUIRE(!ctx->root, H2_ERR_ARG, "not a context created by h2_ctx_create");
    if (!ctx->host_only) {
      dev_set_device(ctx->device);
      for (h2_ctx* c = ctx; c; c = c->aux) dev_sync(c->stream);
    }
    // handles still holding memory of the context keep it until the last
    // of them is destroyed
    ctx_unref(ctx);
  });
}

h2_status h2_tree_build(h2_ctx* ctx, int dim, int64_t n, const double* points, int leaf_size,
                        double eta, h2_tree** out, int64_t* perm_out) {
  return guard([&] {
    H2_REQUIRE(ctx && out && points, H2_ERR_ARG, "NULL argument");
    *out = nullptr;
    H2_REQUIRE(std::isfinite(eta) && eta > 0, H2_ERR_ARG, "eta must be positive");
    auto* t = new h2_tree();
    try {
      t->ct = build_cluster_tree(dim, n, points, leaf_size);
      t->bt = build_block_tree(*t->ct, *t->ct, eta);
      t->eta = eta;
    } catch (...) {
      delete t;
      throw;
    }
    if (perm_out) std::memcpy(perm_out, t->ct->perm.data(), sizeof(int64_t) * n);
    *out = t;
  });
}

h2_status h2_tree_sizes(const h2_tree* tree, int64_t out[7]) {
  return guard([&] {
    H2_REQUIRE(tree && out, H2_ERR_ARG, "NULL argument");
    out[0] = tree->ct->n;
    out[1] = tree->ct->dim;
    out[2] = tree->ct->depth;
    out[3] = tree->ct->ncl;
    out[4] = tree->bt->nblocks();
    out[5] = tree->bt->n_adm;
    out[6] = tree->bt->n_inadm;
  });
}

h2_status h2_tree_structure(const h2_tree* tree, int64_t* cl_off, int64_t* cl_size, int32_t* blk_row,
                            int32_t* blk_col, int8_t* blk_type) {
  return guard([&] {
    H2_REQUIRE(tree, H2_ERR_ARG, "NULL tree");
    const TreeH& T = *tree->ct;
    const BlockTreeH& B = *tree->bt;
    if (cl_off) std::memcpy(cl_off, T.off.data(), sizeof(int64_t) * T.ncl);
    if (cl_size) std::memcpy(cl_size, T.size.data(), sizeof(int64_t) * T.ncl);
    if (blk_row) std::memcpy(blk_row, B.t.data(), sizeof(int32_t) * B.nblocks());
    if (blk_col) std::memcpy(blk_col, B.s.data(), sizeof(int32_t) * B.nblocks());
    if (blk_type)
      for (int b = 0; b < B.nblocks(); ++b) blk_type[b] = B.type[b];
  });
}

static h2_status compress_any(h2_ctx* ctx, const h2_tree* tree, h2_kernel kernel, int order, const double* normals,
                              h2_matrix** out) {
  return guard([&] {
    H2_REQUIRE(out, H2_ERR_ARG, "NULL output");
    *out = nullptr;
    H2_REQUIRE(tree, H2_ERR_ARG, "NULL tree");
    H2_REQUIRE(kernel == H2_K_LOG || kernel == H2_K_EXPNEG || kernel == H2_K_INV4PI || kernel == H2_K_INV ||
                   kernel == H2_K_DLP || kernel == H2_K_POLY2,
               H2_ERR_ARG, "unknown kernel");
    H2_REQUIRE(kernel != H2_K_DLP || normals, H2_ERR_ARG,
               "the double-layer kernel needs normals (h2_compress_kernel_normals)");
    need_device(ctx);
    begin_call(ctx);
    auto* m = new h2_matrix();
    try {
      compress_kernel(ctx, tree, (int)kernel, order, normals, m);
    } catch (...) {
      delete m;
      throw;
    }
    *out = m;
  });
}

h2_status h2_compress_kernel(h2_ctx* ctx, const h2_tree* tree, h2_kernel kernel, int order, h2_matrix** out) {
  return compress_any(ctx, tree, kernel, order, nullptr, out);
}

h2_status h2_compress_kernel_normals(h2_ctx* ctx, const h2_tree* tree, h2_kernel kernel, int order,
                                     const double* normals, h2_matrix** out) {
  if (!normals) {
    g_err = "NULL normals";
    if (out) *out = nullptr;
    return H2_ERR_ARG;
  }
  return compress_any(ctx, tree, kernel, order, normals, out);
}

h2_status h2_mul_intermediate(h2_ctx* ctx, int count, const h2_matrix* const* X, const h2_matrix* const* Y,
                              double eps, h2_precision prec, h2_product** G_out) {
  return guard([&] {
    H2_REQUIRE(G_out && X && Y && count >= 1, H2_ERR_ARG, "bad arguments");
    for (int i = 0; i < count; ++i) {
      G_out[i] = nullptr;
      H2_REQUIRE(X[i] && Y[i], H2_ERR_ARG, "NULL factor");
      H2_REQUIRE(!X[i]->zero && !Y[i]->zero, H2_ERR_ARG,
                 "a factor is a zero matrix (h2_zero_like, not yet filled by h2_recompress)");
    }
    H2_REQUIRE(std::isfinite(eps) && eps >= 0, H2_ERR_ARG, "eps must be >= 0");
    check_precision((int)prec, eps);
    need_device(ctx);
    begin_call(ctx);
    auto one = [&](h2_ctx* c, int i) {
      if (count > 1) rewind_workspaces(c);
      auto* G = new h2_product();
      try {
        phase1(c, X[i], Y[i], eps, (int)prec, G);
      } catch (...) {
        delete G;
        throw;
      }
      G_out[i] = G;
    };
    try {
      if (count == 1 || ctx->root) {
        for (int i = 0; i < count; ++i) one(ctx, i);
      } else {
        std::vector<int64_t> w(count);
        for (int i = 0; i < count; ++i) w[i] = X[i]->c.ct->n;
        run_lanes(ctx, count, w, one);
      }
    } catch (...) {
      for (int j = 0; j < count; ++j) {
        delete G_out[j];
        G_out[j] = nullptr;
      }
      throw;
    }
  });
}

h2_status h2_zero_like(h2_ctx* ctx, const h2_tree* tree, double eta_Z, h2_matrix** Z_out) {
  return guard([&] {
    H2_REQUIRE(Z_out && tree, H2_ERR_ARG, "NULL argument");
    *Z_out = nullptr;
    H2_REQUIRE(!std::isnan(eta_Z) && !std::isinf(eta_Z), H2_ERR_ARG, "eta_Z must be finite");
    need_device(ctx);
    auto* m = new h2_matrix();
    try {
      zero_like(ctx, tree, eta_Z, m);
    } catch (...) {
      delete m;
      throw;
    }
    *Z_out = m;
  });
}

h2_status h2_stats(const void* handle, int kind, h2_stats_t* out) {
  return guard([&] {
    H2_REQUIRE(handle && out, H2_ERR_ARG, "NULL argument");
    H2_REQUIRE(kind == H2_HANDLE_TREE || kind == H2_HANDLE_MATRIX || kind == H2_HANDLE_PRODUCT, H2_ERR_ARG,
               "unknown handle kind");
    handle_stats(handle, kind, out);
  });
}

h2_status h2_export(h2_ctx* ctx, const void* handle, int kind, const char* path) {
  return guard([&] {
    H2_REQUIRE(handle && path, H2_ERR_ARG, "NULL argument");
    H2_REQUIRE(kind == H2_HANDLE_TREE || kind == H2_HANDLE_MATRIX || kind == H2_HANDLE_PRODUCT, H2_ERR_ARG,
               "unknown handle kind");
    if (kind != H2_HANDLE_TREE) need_device(ctx);
    export_handle(ctx, handle, kind, path);
  });
}

h2_status h2_recompress(h2_ctx* ctx, int count, h2_product* const* G, h2_matrix* const* Z, double eps,
                        h2_precision prec) {
  return guard([&] {
    H2_REQUIRE(G && Z && count >= 1, H2_ERR_ARG, "bad arguments");
    for (int i = 0; i < count; ++i) H2_REQUIRE(G[i] && Z[i], H2_ERR_ARG, "NULL operand");
    {
      // the instances run concurrently and each replaces its Z at the end
      std::vector<const h2_matrix*> zs(Z, Z + count);
      std::sort(zs.begin(), zs.end());
      H2_REQUIRE(std::adjacent_find(zs.begin(), zs.end()) == zs.end(), H2_ERR_ARG,
                 "a target Z appears more than once in one call");
    }
    H2_REQUIRE(std::isfinite(eps) && eps >= 0, H2_ERR_ARG, "eps must be >= 0");
    check_precision((int)prec, eps);
    need_device(ctx);
    begin_call(ctx);
    if (count == 1 || ctx->root) {
      for (int i = 0; i < count; ++i) {
        if (count > 1) rewind_workspaces(ctx);
        phase2(ctx, G[i], Z[i], eps, (int)prec);
      }
    } else {
      std::vector<int64_t> w(count);
      for (int i = 0; i < count; ++i) w[i] = G[i]->c.bt ? (int64_t)G[i]->c.bt->nblocks() : 0;
      run_lanes(ctx, count, w, [&](h2_ctx* c, int i) {
        rewind_workspaces(c);
        phase2(c, G[i], Z[i], eps, (int)prec);
      });
    }
  });
}

// [x, x + len) and [y, y + len) share an address
static bool vectors_overlap(const double* x, const double* y, int64_t len) {
  const uintptr_t a = (uintptr_t)x, b = (uintptr_t)y, bytes = (uintptr_t)len * sizeof(double);
  return a < b + bytes && b < a + bytes;
}

h2_status h2_matvec(h2_ctx* ctx, const h2_matrix* A, char op, double alpha, const double* x, double beta,
                    double* y, int nvec) {
  return guard([&] {
    H2_REQUIRE(A && x && y && nvec >= 1, H2_ERR_ARG, "bad arguments");
    H2_REQUIRE(op == 'N' || op == 'T', H2_ERR_ARG, "op must be 'N' or 'T'");
    H2_REQUIRE(!vectors_overlap(x, y, A->c.ct->n * (int64_t)nvec), H2_ERR_ARG, "x and y overlap");
    need_device(ctx);
    begin_call(ctx);
    matvec(ctx, A->c, op == 'T', alpha, x, beta, y, nvec);
  });
}

h2_status h2_matvec_noalloc(h2_ctx* ctx, const h2_matrix* A, char op, double alpha, const double* x,
                            double beta, double* y, int nvec) {
  return guard([&] {
    H2_REQUIRE(A && x && y && nvec >= 1, H2_ERR_ARG, "bad arguments");
    H2_REQUIRE(op == 'N' || op == 'T', H2_ERR_ARG, "op must be 'N' or 'T'");
    H2_REQUIRE(!vectors_overlap(x, y, A->c.ct->n * (int64_t)nvec), H2_ERR_ARG, "x and y overlap");
    need_device(ctx);
    begin_call(ctx);
    matvec_noalloc(ctx, A->c, op == 'T', alpha, x, beta, y, nvec);
  });
}

h2_status h2_product_matvec(h2_ctx* ctx, const h2_product* G, char op, double alpha, const double* x,
                            double beta, double* y, int nvec) {
  return guard([&] {
    H2_REQUIRE(G && x && y && nvec >= 1, H2_ERR_ARG, "bad arguments");
    H2_REQUIRE(op == 'N' || op == 'T', H2_ERR_ARG, "op must be 'N' or 'T'");
    H2_REQUIRE(!vectors_overlap(x, y, G->c.ct->n * (int64_t)nvec), H2_ERR_ARG, "x and y overlap");
    need_device(ctx);
    begin_call(ctx);
    matvec(ctx, G->c, op == 'T', alpha, x, beta, y, nvec);
  });
}

h2_status h2_to_dense(h2_ctx* ctx, const h2_matrix* A, double* out, int64_t ld) {
  return guard([&] {
    H2_REQUIRE(A && out && ld >= A->c.ct->n, H2_ERR_ARG, "bad arguments");
    need_device(ctx);
    begin_call(ctx);
    to_dense(ctx, A->c, out, ld);
  });
}

h2_status h2_product_to_dense(h2_ctx* ctx, const h2_product* G, double* out, int64_t ld) {
  return guard([&] {
    H2_REQUIRE(G && out && ld >= G->c.ct->n, H2_ERR_ARG, "bad arguments");
    need_device(ctx);
    begin_call(ctx);
    to_dense(ctx, G->c, out, ld);
  });
}

h2_status h2_matrix_basis(h2_ctx* ctx, const h2_matrix* A, int which, int cluster, double* out, int64_t ld) {
  return guard([&] {
    H2_REQUIRE(A && out && (which == 0 || which == 1), H2_ERR_ARG, "bad arguments");
    need_device(ctx);
    begin_call(ctx);
    basis_dense(ctx, A->c, which, cluster, out, ld);
  });
}

h2_status h2_product_basis(h2_ctx* ctx, const h2_product* G, int which, int cluster, double* out, int64_t ld) {
  return guard([&] {
    H2_REQUIRE(G && out && (which == 0 || which == 1), H2_ERR_ARG, "bad arguments");
    need_device(ctx);
    begin_call(ctx);
    basis_dense(ctx, G->c, which, cluster, out, ld);
  });
}

h2_status h2_matrix_ranks(const h2_matrix* A, int which, int32_t* out) {
  return guard([&] {
    H2_REQUIRE(A && out && (which == 0 || which == 1), H2_ERR_ARG, "bad arguments");
    const auto& r = which == 0 ? A->c.V.rank : A->c.W.rank;
    std::memcpy(out, r.data(), sizeof(int32_t) * r.size());
  });
}

h2_status h2_product_ranks(const h2_product* G, int which, int32_t* out) {
  return guard([&] {
    H2_REQUIRE(G && out && (which == 0 || which == 1), H2_ERR_ARG, "bad arguments");
    const auto& r = which == 0 ? G->c.V.rank : G->c.W.rank;
    std::memcpy(out, r.data(), sizeof(int32_t) * r.size());
  });
}

h2_status h2_product_sizes(const h2_product* G, int64_t out[5]) {
  return guard([&] {
    H2_REQUIRE(G && out, H2_ERR_ARG, "bad arguments");
    out[0] = G->c.bt->nblocks();
    out[1] = G->c.bt->n_adm;
    out[2] = G->c.bt->n_inadm;
    out[3] = G->n_triples;
    out[4] = (int64_t)(G->mem.total + G->mem_aux.total + G->mem_nf.total);
  });
}

int h2_step_times(h2_ctx* ctx, double* out, int n, int reset) {
  if (!ctx || !out) return 0;
  if (!ctx->host_only) {
    try {
      dev_set_device(ctx->device);
      steps_collect(ctx);
      aux_collect(ctx);
    } catch (...) {
      return 0;
    }
  }
  int m = std::min(n, 16);
  for (int i = 0; i < m; ++i) out[i] = i < 8 ? ctx->step_ms[i] : ctx->host_ms[i - 8];
  if (reset) {
    for (double& v : ctx->step_ms) v = 0.0;
    for (double& v : ctx->host_ms) v = 0.0;
  }
  return m;
}

h2_status h2_set_rank_rule(h2_ctx* ctx, int rule) {
  return guard([&] {
    H2_REQUIRE(ctx, H2_ERR_ARG, "NULL context");
    H2_REQUIRE(rule == H2_RANK_ABS || rule == H2_RANK_REL_FROB, H2_ERR_ARG, "unknown rank rule");
    ctx->rank_rule = rule;
  });
}

h2_status h2_set_level_factor(h2_ctx* ctx, double zeta) {
  return guard([&] {
    H2_REQUIRE(ctx, H2_ERR_ARG, "NULL context");
    H2_REQUIRE(zeta > 0.0 && zeta <= 1.0, H2_ERR_ARG, "level factor outside (0, 1]");
    ctx->level_factor = zeta;
  });
}

h2_status h2_set_run_scratch(h2_ctx* ctx, int64_t bytes) {
  return guard([&] {
    H2_REQUIRE(ctx, H2_ERR_ARG, "NULL context");
    ctx->run_scratch = bytes <= 0 ? kRunScratchDefault : (size_t)bytes;
  });
}

h2_status h2_debug_fail_after(h2_ctx* ctx, int launches) {
  return guard([&] {
    H2_REQUIRE(ctx, H2_ERR_ARG, "NULL context");
    ctx->fail_after = launches < 0 ? -1 : launches;
  });
}

h2_status h2_profile(h2_ctx* ctx, int families) {
  return guard([&] {
    H2_REQUIRE(ctx, H2_ERR_ARG, "NULL context");
    ctx->profile = families & ((1 << h2::KK_COUNT) - 1);
  });
}

h2_status h2_kernel_stats(h2_ctx* ctx, int kind, double out[4], int reset) {
  return guard([&] {
    H2_REQUIRE(ctx && out && kind >= 0 && kind < KK_COUNT, H2_ERR_ARG, "bad arguments");
    if (!ctx->host_only) {
      dev_set_device(ctx->device);
      kernel_stats_collect(ctx);
    }
    const KernelStat& k = ctx->kstat[kind];
    out[0] = k.ms;
    out[1] = (double)k.launches;
    out[2] = k.flops;
    out[3] = k.bytes;
    if (reset)
      for (auto& s : ctx->kstat) s = KernelStat{};
  });
}

void h2_tree_destroy(h2_tree* tree) { delete tree; }
void h2_matrix_destroy(h2_matrix* A) { delete A; }
void h2_product_destroy(h2_product* G) { delete G; }

}  // extern "C"
