// Runtime: errors, device arenas with a chunk cache, pinned staging of
// launch descriptors, step timers and the batched launch builders.
#include <cmath>

#include "internal.h"

namespace h2 {

[[noreturn]] void fail(h2_status c, const std::string& msg) { throw Error(c, msg); }

// ---------------------------------------------------------------------------
// arenas: bump allocation in device chunks; chunks return to the context cache
// ---------------------------------------------------------------------------
static constexpr size_t kChunk = (size_t)64 << 20;

static h2_ctx* root_of(h2_ctx* c) { return c->root ? c->root : c; }

// index of the smallest chunk of `v` with at least `bytes`, or -1
static int smallest_fit(const std::vector<std::pair<char*, size_t>>& v, size_t bytes) {
  size_t best = (size_t)-1;
  int bi = -1;
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i].second >= bytes && v[i].second < best) {
      best = v[i].second;
      bi = (int)i;
    }
  return bi;
}

// the root pool's chunks back to the allocator; false if it was empty
static bool pool_flush(h2_ctx* root) {
  std::lock_guard<std::mutex> lock(root->pool_mu);
  if (root->pool.empty()) return false;
  for (auto& c : root->pool) ctx_free(root, c.first);
  root->pool.clear();
  return true;
}

void* ctx_malloc(h2_ctx* ctx, size_t bytes) {
  if (ctx && ctx->alloc_fn) {
    void* p = ctx->alloc_fn(bytes, ctx->alloc_user);
    H2_REQUIRE(p, H2_ERR_ALLOC, "the allocator callback returned NULL for " + std::to_string(bytes) + " bytes");
    return p;
  }
  return dev_malloc(bytes);
}

void ctx_free(h2_ctx* ctx, void* p) {
  if (!p) return;
  if (ctx && ctx->free_fn)
    ctx->free_fn(p, ctx->alloc_user);
  else
    dev_free(p);
}

void* Arena::alloc(size_t bytes) {
  bytes = (bytes + 255) & ~(size_t)255;
  if (bytes == 0) bytes = 256;
  if (fixed) {
    H2_REQUIRE(fixed_used + bytes <= fixed_cap, H2_ERR_ARG,
               "the call needs more than the fixed scratch of " + std::to_string(fixed_cap) + " bytes");
    void* p = fixed + fixed_used;
    fixed_used += bytes;
    return p;
  }
  while (cur < chunks.size()) {
    if (used + bytes <= chunks[cur].second) {
      void* p = chunks[cur].first + used;
      used += bytes;
      return p;
    }
    ++cur;
    used = 0;
  }
  // the smallest chunk that fits from the context's own cache, else from
  // the family's pool, else a new one (after handing the pool back to the
  // allocator if the first attempt fails)
  if (ctx) {
    std::lock_guard<std::mutex> lock(ctx->ret_mu);
    for (auto& c : ctx->returned) ctx->cache.push_back(c);
    ctx->returned.clear();
  }
  std::pair<char*, size_t> ch{nullptr, 0};
  if (ctx) {
    const int bi = smallest_fit(ctx->cache, bytes);
    if (bi >= 0) {
      ch = ctx->cache[bi];
      ctx->cache.erase(ctx->cache.begin() + bi);
    }
  }
  if (!ch.first && ctx) {
    h2_ctx* r = root_of(ctx);
    std::lock_guard<std::mutex> lock(r->pool_mu);
    const int bi = smallest_fit(r->pool, bytes);
    if (bi >= 0) {
      ch = r->pool[bi];
      r->pool.erase(r->pool.begin() + bi);
    }
  }
  if (!ch.first) {
    const size_t sz = std::max(bytes, kChunk);
    try {
      ch = {(char*)ctx_malloc(ctx, sz), sz};
    } catch (const Error&) {
      if (!ctx || !pool_flush(root_of(ctx))) throw;
      ch = {(char*)ctx_malloc(ctx, sz), sz};
    }
  }
  chunks.push_back(ch);
  cur = chunks.size() - 1;
  used = bytes;
  total += ch.second;
  return ch.first;
}

void Arena::release() {
  if (ctx) {
    std::lock_guard<std::mutex> lock(ctx->ret_mu);
    for (auto& c : chunks) ctx->returned.push_back(c);
  } else {
    for (auto& c : chunks) dev_free(c.first);
  }
  chunks.clear();
  cur = used = total = 0;
}

void pool_idle_memory(h2_ctx* root) {
  std::vector<h2_ctx*> fam;
  for (h2_ctx* c = root; c; c = c->aux) fam.push_back(c);
  for (h2_ctx* l : root->lanes)
    for (h2_ctx* c = l; c; c = c->aux) fam.push_back(c);
  for (h2_ctx* c : fam) {
    c->ws.release();
    std::vector<std::pair<char*, size_t>> idle;
    {
      std::lock_guard<std::mutex> lock(c->ret_mu);
      idle.swap(c->returned);
    }
    idle.insert(idle.end(), c->cache.begin(), c->cache.end());
    c->cache.clear();
    std::lock_guard<std::mutex> lock(root->pool_mu);
    root->pool.insert(root->pool.end(), idle.begin(), idle.end());
  }
}

void rewind_workspaces(h2_ctx* ctx) {
  for (h2_ctx* c = ctx; c; c = c->aux) c->ws.reset();
}

void Arena::bind(h2_ctx* c) {
  if (ctx == c) return;
  H2_REQUIRE(chunks.empty(), H2_ERR_ARG, "a handle's memory cannot move to another context");
  h2_ctx* o = root_of(c);
  o->refs.fetch_add(1);
  if (owner) ctx_unref(owner);
  ctx = c;
  owner = o;
}

Arena::~Arena() {
  release();
  if (owner) ctx_unref(owner);
}

void ctx_unref(h2_ctx* root) {
  if (root->refs.fetch_sub(1) == 1) delete root;
}

double* zeros(h2_ctx* ctx, Arena& a, size_t count) {
  double* p = a.get<double>(count);
  dev_zero(p, count * sizeof(double), ctx->stream);
  return p;
}

// ---------------------------------------------------------------------------
// descriptor uploads through pinned staging
// ---------------------------------------------------------------------------
char* stage_alloc(h2_ctx* ctx, size_t bytes) {
  size_t need = (bytes + 255) & ~(size_t)255;
  if (ctx->stage_used + need > ctx->stage_cap) {
    dev_sync(ctx->stream);  // earlier copies out of the staging buffer are done
    ctx->stage_used = 0;
    if (ctx->no_alloc) {  // the staging is reused as it is, never reallocated
      H2_REQUIRE(need <= ctx->stage_cap, H2_ERR_ARG,
                 "a descriptor table exceeds the context's staging (" + std::to_string(ctx->stage_cap) + " bytes)");
      char* h = ctx->stage;
      ctx->stage_used = need;
      return h;
    }
    // a call that fills the staging waits here: the buffer grows (up to
    // 1 GiB) so that later calls of the same size do not
    constexpr size_t kStageMax = (size_t)1 << 30;
    if (need > ctx->stage_cap || ctx->stage_cap < kStageMax) {
      dev_free_host(ctx->stage);
      ctx->stage = ctx->stage_dev = nullptr;
      ctx->stage_cap = std::max(need, std::min(ctx->stage_cap * 2, kStageMax));
      ctx->stage = (char*)dev_malloc_host(ctx->stage_cap);
      ctx->stage_dev = (char*)dev_host_view(ctx->stage);
    }
  }
  char* h = ctx->stage + ctx->stage_used;
  ctx->stage_used += need;
  return h;
}

void* stage_upload(h2_ctx* ctx, const char* h, size_t bytes) {
  void* d = ctx->ws.alloc(bytes);
  if (ctx->stage_dev)
    dev_pull(d, ctx->stage_dev + (h - ctx->stage), bytes, ctx->stream);
  else
    dev_h2d(d, h, bytes, ctx->stream);
  return d;
}

// Descriptor tables read only by the launch that follows: a small table is
// read by the kernel straight from the mapped staging (no copy launch); the
// staging is reused only after the stream has been synchronised, which the
// launch precedes.  Larger tables are copied into the workspace.
static constexpr size_t kStageViewMax = (size_t)32 << 10;
void* stage_launch(h2_ctx* ctx, const char* h, size_t bytes) {
  if (ctx->stage_dev && bytes <= kStageViewMax) return ctx->stage_dev + (h - ctx->stage);
  return stage_upload(ctx, h, bytes);
}

void* upload_launch_bytes(h2_ctx* ctx, const void* src, size_t bytes) {
  char* h = stage_alloc(ctx, bytes);
  std::memcpy(h, src, bytes);
  return stage_launch(ctx, h, bytes);
}

void* upload_bytes(h2_ctx* ctx, const void* src, size_t bytes) {
  char* h = stage_alloc(ctx, bytes);
  std::memcpy(h, src, bytes);
  return stage_upload(ctx, h, bytes);
}

const int32_t* read_back(h2_ctx* ctx, const int32_t* dev, int n) {
  int32_t* h = (int32_t*)stage_alloc(ctx, sizeof(int32_t) * std::max(n, 1));
  if (ctx->stage_dev)
    dev_push_i32((int32_t*)(ctx->stage_dev + ((char*)h - ctx->stage)), dev, n, ctx->stream);
  else
    dev_d2h(h, dev, sizeof(int32_t) * n, ctx->stream);
  return h;
}

void ctx_sync(h2_ctx* ctx) {
  dev_sync(ctx->stream);
  ctx->stage_used = 0;
}

// ---------------------------------------------------------------------------
// step timers
// ---------------------------------------------------------------------------
void step_begin(h2_ctx* ctx, int step) {
  // the intervals are resolved when they are read; a long run of calls
  // without a read resolves them here (this waits for the stream)
  if (ctx->events.size() > 4096) steps_collect(ctx);
  ctx->host_t0[step] = std::chrono::steady_clock::now();
  void* e = pool_event(ctx);
  dev_event_record(e, ctx->stream);
  ctx->events.push_back(e);
  ctx->ev_step.push_back(-1 - step);
}
void step_end(h2_ctx* ctx, int step) {
  ctx->host_ms[step] +=
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - ctx->host_t0[step]).count();
  void* e = pool_event(ctx);
  dev_event_record(e, ctx->stream);
  ctx->events.push_back(e);
  ctx->ev_step.push_back(step);
}
void steps_collect(h2_ctx* ctx) {
  for (size_t i = 0; i + 1 < ctx->events.size(); ++i) {
    int s = ctx->ev_step[i];
    if (s < 0 && ctx->ev_step[i + 1] == -1 - s)
      ctx->step_ms[-1 - s] += dev_event_ms(ctx->events[i], ctx->events[i + 1]);
  }
  for (void* e : ctx->events) ctx->ev_pool.push_back(e);
  ctx->events.clear();
  ctx->ev_step.clear();
}

// ---------------------------------------------------------------------------
// launch timers: one pair of events per launch, resolved at collection
// ---------------------------------------------------------------------------
void* pool_event(h2_ctx* ctx) {
  if (ctx->ev_pool.empty()) return dev_event_create();
  void* e = ctx->ev_pool.back();
  ctx->ev_pool.pop_back();
  return e;
}

LaunchTimer::LaunchTimer(h2_ctx* c, int k, double f, double b) : ctx(c), kind(k), flops(f), bytes(b) {
  if (ctx->fail_after >= 0 && ctx->fail_after-- == 0) fail(H2_ERR_DEVICE, "injected failure before a launch");
  if (!((ctx->profile >> kind) & 1) || ctx->no_alloc) return;  // events are not created there
  a = pool_event(ctx);
  dev_event_record(a, ctx->stream);
}

LaunchTimer::~LaunchTimer() {
  if (!a) return;
  void* b = pool_event(ctx);
  dev_event_record(b, ctx->stream);
  PendingLaunch p{a, b, kind, flops, bytes};
  p.work = work;
  p.nwork = nwork;
  ctx->pending.push_back(p);
}

WorkCounts work_counts(h2_ctx* ctx, int n, int kind) {
  WorkCounts w;
  if (!((ctx->profile >> kind) & 1) || n <= 0 || ctx->no_alloc) return w;
  w.n = n;
  w.dev = ctx->ws.get<double>(n);
  if (ctx->prof_host.empty() || ctx->prof_used + n > ctx->prof_chunk) {
    size_t cap = std::max<size_t>(n, 1 << 18);
    ctx->prof_host.push_back({(double*)dev_malloc_host(cap * sizeof(double)), cap});
    ctx->prof_chunk = cap;
    ctx->prof_used = 0;
  }
  w.host = ctx->prof_host.back().first + ctx->prof_used;
  ctx->prof_used += n;
  return w;
}

// ---------------------------------------------------------------------------
// auxiliary context: the column passes run on it concurrently with the row
// passes (own stream, workspace, staging, events; same device)
// ---------------------------------------------------------------------------
static h2_ctx* side_ctx(h2_ctx* ctx) {
  auto* a = new h2_ctx();
  a->device = ctx->device;
  a->host_only = false;
  a->ws.ctx = a;
  a->root = root_of(ctx);
  a->alloc_fn = ctx->alloc_fn;
  a->free_fn = ctx->free_fn;
  a->alloc_user = ctx->alloc_user;
  a->scratch_dev = ctx->scratch_dev;
  try {
    a->stream = dev_stream_create();
    a->own_stream = true;
    a->stage_cap = (size_t)16 << 20;
    a->stage = (char*)dev_malloc_host(a->stage_cap);
    a->stage_dev = (char*)dev_host_view(a->stage);
  } catch (...) {
    delete a;
    throw;
  }
  return a;
}

h2_ctx* lane_ctx(h2_ctx* ctx, int w) {
  H2_REQUIRE(w >= 0 && w < kBatchLanes && !ctx->root, H2_ERR_ARG, "lane of a non-root context");
  if ((int)ctx->lanes.size() <= w) ctx->lanes.resize(w + 1, nullptr);
  if (!ctx->lanes[w]) ctx->lanes[w] = side_ctx(ctx);
  return ctx->lanes[w];
}

h2_ctx* aux_ctx(h2_ctx* ctx) {
  if (!ctx->aux) ctx->aux = side_ctx(ctx);
  return ctx->aux;
}

AuxRun::AuxRun(h2_ctx* c, std::function<void(h2_ctx*)> f) : AuxRun(c, aux_ctx(c), std::move(f)) {}

AuxRun::AuxRun(h2_ctx* c, h2_ctx* a_, std::function<void(h2_ctx*)> f) : ctx(c), aux(a_) {
  aux->profile = ctx->profile;
  aux->prec = ctx->prec;
  aux->rank_rule = ctx->rank_rule;
  aux->level_factor = ctx->level_factor;
  aux->run_scratch = ctx->run_scratch;
  // the staging of the previous run is free once that run's work is done
  // (usually long ago): wait for its end event, not for the stream, which is
  // about to wait for ctx's queue
  if (aux->drain) {
    dev_event_sync(aux->drain);
    aux->stage_used = 0;
  }
  void* e = pool_event(ctx);
  dev_event_record(e, ctx->stream);
  dev_stream_wait(aux->stream, e);  // the wait takes the event as recorded now
  ctx->ev_pool.push_back(e);
  const int dev = ctx->device;
  h2_ctx* a = aux;
  th = std::thread([this, f, dev, a] {
    try {
      dev_set_device(dev);  // the current device is per host thread
      f(a);
    } catch (...) {
      err = std::current_exception();
    }
  });
}

void AuxRun::join() {
  joined = true;
  if (th.joinable()) th.join();
  if (!aux->drain) aux->drain = dev_event_create();
  dev_event_record(aux->drain, aux->stream);
  dev_stream_wait(ctx->stream, aux->drain);
  if (err) {
    std::exception_ptr x = err;
    err = nullptr;
    std::rethrow_exception(x);
  }
}

// Error path (join() not reached because the owning thread threw): the
// auxiliary thread has issued work that may still run on the device, reading
// workspace and staging that the next call on these contexts reuses.  Order
// the context stream after it and wait for it before the exception leaves.
AuxRun::~AuxRun() {
  if (th.joinable()) th.join();
  if (joined) return;
  try {
    if (!aux->drain) aux->drain = dev_event_create();
    dev_event_record(aux->drain, aux->stream);
    dev_stream_wait(ctx->stream, aux->drain);
    dev_sync(aux->stream);
    aux->stage_used = 0;
  } catch (...) {
  }
}

void aux_collect(h2_ctx* ctx) {
  std::vector<h2_ctx*> side = ctx->lanes;
  side.push_back(ctx->aux);
  for (h2_ctx* a : side) {
    if (!a) continue;
    aux_collect(a);  // the side context's own ones first
    steps_collect(a);
    for (int i = 0; i < 8; ++i) {
      ctx->step_ms[i] += a->step_ms[i];
      ctx->host_ms[i] += a->host_ms[i];
      a->step_ms[i] = 0.0;
      a->host_ms[i] = 0.0;
    }
  }
}

void kernel_stats_collect(h2_ctx* ctx) {
  std::vector<h2_ctx*> side = ctx->lanes;
  side.push_back(ctx->aux);
  for (h2_ctx* a : side) {
    if (!a) continue;
    kernel_stats_collect(a);
    for (int k = 0; k < KK_COUNT; ++k) {
      ctx->kstat[k].ms += a->kstat[k].ms;
      ctx->kstat[k].flops += a->kstat[k].flops;
      ctx->kstat[k].bytes += a->kstat[k].bytes;
      ctx->kstat[k].launches += a->kstat[k].launches;
      a->kstat[k] = KernelStat{};
    }
  }
  for (auto& p : ctx->pending) {
    KernelStat& k = ctx->kstat[p.kind];
    k.ms += dev_event_ms(p.a, p.b);
    k.launches += 1;
    if (p.work) {  // the copy of the counts follows the end event on the stream
      dev_sync(ctx->stream);
      double f = 0;
      for (int i = 0; i < p.nwork; ++i) f += p.work[i];
      k.flops += f;
    } else {
      k.flops += p.flops;
    }
    k.bytes += p.bytes;
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.clear();
  // pinned count chunks are reused once nothing refers to them
  if (ctx->prof_host.size() > 1) {
    for (size_t i = 0; i + 1 < ctx->prof_host.size(); ++i) dev_free_host(ctx->prof_host[i].first);
    ctx->prof_host.erase(ctx->prof_host.begin(), ctx->prof_host.end() - 1);
  }
  ctx->prof_used = 0;
}

// ---------------------------------------------------------------------------
// batch builders
// ---------------------------------------------------------------------------
void GemmBatch::out(double* C, int64_t ldc, int m, int n, bool accumulate) {
  GemmOut o{};
  o.C = C;
  o.ldc = std::max<int64_t>(ldc, 1);
  o.m = m;
  o.n = n;
  o.t0 = o.t1 = (int32_t)terms.size();
  o.beta = accumulate ? 1 : 0;
  outs.push_back(o);
}

void GemmBatch::term(const double* A, int64_t lda, bool tA, const double* B, int64_t ldb, bool tB,
                     int k, double alpha, const double* scale, int scale_mode) {
  GemmTerm t{};
  t.A = A;
  t.B = B;
  t.lda = std::max<int64_t>(lda, 1);
  t.ldb = std::max<int64_t>(ldb, 1);
  t.k = k;
  t.flags = (tA ? GT_TA : 0) | (tB ? GT_TB : 0) |
            (scale ? (scale_mode == 2 ? GT_SCALE_INV : GT_SCALE_MUL) : 0);
  t.scale = scale;
  t.alpha = alpha;
  if (k <= 0) return;  // empty contraction contributes nothing
  terms.push_back(t);
  outs.back().t1 = (int32_t)terms.size();
}

void GemmBatch::copy(const double* A, int64_t lda, bool tA, int k, double alpha, const double* scale,
                     int scale_mode) {
  term(A, lda, tA, nullptr, 1, false, k, alpha, scale, scale_mode);
  if (k > 0) terms.back().flags |= GT_BEYE;
}

void GemmBatch::run(h2_ctx* ctx) {
  bool any = false;
  for (const GemmOut& o : outs)
    if (o.m > 0 && o.n > 0 && !(o.t0 == o.t1 && o.beta)) {
      any = true;
      break;
    }
  if (!any) {
    outs.clear();
    terms.clear();
    return;
  }
  // outputs and terms written straight into pinned staging, one copy; the
  // kernel deals each output's tiles to its own workgroup, or, when some
  // output has more than kGemmTilesPerGroup tiles, to one workgroup per run
  // of that many tiles (a list of output / first-tile pairs)
  int64_t ngroups = 0;
  bool split = false;
  for (const GemmOut& o : outs) {
    const int64_t tiles = (int64_t)((std::max(o.m, 0) + 15) / 16) * ((std::max(o.n, 0) + 15) / 16);
    ngroups += std::max<int64_t>(1, (tiles + kGemmTilesPerGroup - 1) / kGemmTilesPerGroup);
    split = split || tiles > kGemmTilesPerGroup;
  }
  const size_t so = outs.size() * sizeof(GemmOut), st = std::max<size_t>(terms.size(), 1) * sizeof(GemmTerm);
  const size_t o_t = (so + 255) & ~(size_t)255, o_w = o_t + ((st + 255) & ~(size_t)255);
  const size_t sw = split ? (size_t)ngroups * 2 * sizeof(int32_t) : 0;
  char* h = stage_alloc(ctx, o_w + sw);
  std::memcpy(h, outs.data(), so);
  if (!terms.empty()) std::memcpy(h + o_t, terms.data(), terms.size() * sizeof(GemmTerm));
  if (split) {
    int32_t* w = (int32_t*)(h + o_w);
    for (size_t i = 0; i < outs.size(); ++i) {
      const GemmOut& o = outs[i];
      const int tiles = ((std::max(o.m, 0) + 15) / 16) * ((std::max(o.n, 0) + 15) / 16);
      for (int t0 = 0; t0 < std::max(tiles, 1); t0 += kGemmTilesPerGroup) {
        *w++ = (int32_t)i;
        *w++ = t0;
      }
    }
  }
  char* dev = (char*)stage_launch(ctx, h, o_w + sw);
  // algorithmic work: 2 m n k per term; bytes: operands read once, C written
  double flops = 0, bytes = 0;
  const double es = prec ? 4.0 : 8.0;
  for (const GemmOut& o : outs) {
    if (o.m <= 0 || o.n <= 0) continue;
    bytes += es * (double)o.m * o.n * (o.beta ? 2 : 1);
    for (int q = o.t0; q < o.t1; ++q) {
      const GemmTerm& t = terms[q];
      flops += (t.flags & GT_BEYE) ? 0.0 : 2.0 * o.m * o.n * t.k;
      bytes += es * ((double)o.m * t.k + ((t.flags & GT_BEYE) ? 0.0 : (double)t.k * o.n));
    }
  }
  LaunchTimer lt(ctx, KK_GEMM, flops, bytes);
  k_gemm_sum((GemmOut*)dev, (GemmTerm*)(dev + o_t), split ? (int32_t*)(dev + o_w) : nullptr,
             split ? (int)ngroups : (int)outs.size(), prec, ctx->stream);
  outs.clear();
  terms.clear();
}

void Chain3Batch::add(double* C, int64_t ldc, int m, int n, const double* A, int64_t lda, bool tA, int p,
                      const double* B, int64_t ldb, int q, const double* D, int64_t ldd, bool dT,
                      bool accumulate) {
  H2_REQUIRE(fits(m, n, p, q), H2_ERR_ARG, "chained product: dimension over 64");
  if (m <= 0 || n <= 0) return;
  if ((p <= 0 || q <= 0) && accumulate) return;  // adds nothing
  Chain3 c{};
  c.C = C;
  c.ldc = std::max<int64_t>(ldc, 1);
  c.m = m;
  c.n = n;
  c.A = A;
  c.lda = std::max<int64_t>(lda, 1);
  c.tA = tA ? 1 : 0;
  c.p = std::max(p, 0);
  c.B = B;
  c.ldb = std::max<int64_t>(ldb, 1);
  c.q = std::max(q, 0);
  c.D = D;
  c.ldd = std::max<int64_t>(ldd, 1);
  c.dT = dT ? 1 : 0;
  c.beta = accumulate ? 1 : 0;
  items.push_back(c);
}

void Chain3Batch::run(h2_ctx* ctx) {
  if (items.empty()) return;
  double flops = 0, bytes = 0;
  for (const Chain3& c : items) {
    flops += 2.0 * c.m * c.p * c.q + 2.0 * c.m * c.q * c.n;
    bytes += 8.0 * ((double)c.m * c.p + (double)c.p * c.q + (double)c.n * c.q + (double)c.m * c.n * (c.beta ? 2 : 1));
  }
  Chain3* d = upload_launch(ctx, items);
  LaunchTimer lt(ctx, KK_GEMM, flops, bytes);
  k_chain3(d, (int)items.size(), ctx->stream);
  items.clear();
}

void TriBatch::out(double* C, int64_t ldc, int m, int n, int q0, int q1, bool accumulate) {
  if (m <= 0 || n <= 0) return;
  const int bs = block ? 64 : std::max(m, n);
  for (int i0 = 0; i0 < m; i0 += bs)
    for (int j0 = 0; j0 < n; j0 += bs) {
      TriOut o{};
      o.C = C + i0 + (int64_t)j0 * std::max<int64_t>(ldc, 1);
      o.ldc = std::max<int64_t>(ldc, 1);
      o.m = std::min(bs, m - i0);
      o.n = std::min(bs, n - j0);
      o.q0 = q0;
      o.q1 = q1;
      o.beta = accumulate ? 1 : 0;
      o.ro = i0;
      o.co = j0;
      outs.push_back(o);
    }
}

void TriBatch::run(h2_ctx* ctx, double flops) {
  if (outs.empty()) return;
  if (block) {
    for (const TriOut& o : outs) H2_REQUIRE(o.m <= 64 && o.n <= 64, H2_ERR_ARG, "triple block product: output over 64 x 64");
    double bytes = 0;
    for (const TriOut& o : outs) bytes += 8.0 * o.m * o.n * (o.beta ? 2 : 1);
    TriOut* d = upload_launch(ctx, outs);
    LaunchTimer lt(ctx, KK_GEMM, flops, bytes);
    k_gemm_tri_block(d, (int)outs.size(), fam, prec, ctx->stream);
    outs.clear();
    return;
  }
  size_t ntiles = 0;
  for (const TriOut& o : outs) ntiles += (size_t)((o.m + 15) / 16) * ((o.n + 15) / 16);
  const size_t so = outs.size() * sizeof(TriOut), o_t = (so + 255) & ~(size_t)255;
  char* h = stage_alloc(ctx, o_t + ntiles * 3 * sizeof(int32_t));
  std::memcpy(h, outs.data(), so);
  int32_t* tl = (int32_t*)(h + o_t);
  for (size_t i = 0; i < outs.size(); ++i)
    for (int j0 = 0; j0 < outs[i].n; j0 += 16)
      for (int i0 = 0; i0 < outs[i].m; i0 += 16) {
        *tl++ = (int32_t)i;
        *tl++ = i0;
        *tl++ = j0;
      }
  char* dev = (char*)stage_launch(ctx, h, o_t + ntiles * 3 * sizeof(int32_t));
  double bytes = 0;
  for (const TriOut& o : outs) bytes += 8.0 * o.m * o.n * (o.beta ? 2 : 1);
  LaunchTimer lt(ctx, KK_GEMM, flops, bytes);
  k_gemm_tri((TriOut*)dev, (int32_t*)(dev + o_t), (int)ntiles, fam, prec, ctx->stream);
  outs.clear();
}

void QrBatch::add(double* A, int64_t lda, int m, int n, double* tau, double* R, int64_t ldr, int rrows) {
  if (m <= 0 || n <= 0) return;
  QrProb q{};
  q.A = A;
  q.lda = std::max<int64_t>(lda, 1);
  q.m = m;
  q.n = n;
  q.tau = tau;
  q.R = R;
  q.ldr = std::max<int64_t>(ldr, 1);
  q.rrows = rrows;
  p.push_back(q);
}

// dynamic LDS of a launch: the largest working set that fits the device limit
static int lds_for(size_t largest_fitting) { return (int)std::max<size_t>(largest_fitting, 1); }

void QrBatch::run(h2_ctx* ctx) {
  if (p.empty()) return;
  const size_t lim = (size_t)lds_limit_doubles();
  size_t lds = 0;
  double flops = 0, bytes = 0;
  for (const QrProb& q : p) {
    size_t need = qr_need_doubles(q.m, q.n);
    if (need <= lim) lds = std::max(lds, need);
    double m = q.m, n = q.n, r = std::min(m, n);
    flops += 2.0 * m * n * r - (m + n) * r * r + 2.0 * r * r * r / 3.0;
    bytes += 16.0 * m * n;
  }
  QrProb* d = upload_launch(ctx, p);
  LaunchTimer lt(ctx, KK_TSQR, flops, bytes);
  k_qr(d, (int)p.size(), lds_for(lds), ctx->stream);
  p.clear();
}

void ApplyBatch::add(const double* V, int64_t ldv, const double* tau, int m, int nrefl, double* C,
                     int64_t ldc, int ncols, bool trans) {
  if (m <= 0 || nrefl <= 0 || ncols <= 0) return;
  ApplyProb a{};
  a.V = V;
  a.ldv = std::max<int64_t>(ldv, 1);
  a.tau = tau;
  a.m = m;
  a.nrefl = nrefl;
  a.C = C;
  a.ldc = std::max<int64_t>(ldc, 1);
  a.ncols = ncols;
  a.trans = trans ? 1 : 0;
  p.push_back(a);
}

void ApplyBatch::run(h2_ctx* ctx) {
  if (p.empty()) return;
  const size_t lim = (size_t)lds_limit_doubles();
  size_t lds = 0;
  std::vector<int32_t> work;
  double flops = 0, bytes = 0;
  for (size_t i = 0; i < p.size(); ++i) {
    size_t need = (size_t)p[i].m * p[i].nrefl;
    if (need <= lim) lds = std::max(lds, need);
    for (int c = 0; c < p[i].ncols; c += 64) {
      work.push_back((int32_t)i);
      work.push_back(c);
    }
    flops += 4.0 * p[i].m * p[i].nrefl * p[i].ncols;
    bytes += 16.0 * p[i].m * p[i].ncols;
  }
  // one staging region for both tables (the launch reads them together)
  const size_t sp = p.size() * sizeof(ApplyProb), o_w = (sp + 255) & ~(size_t)255;
  const size_t sw = work.size() * sizeof(int32_t);
  char* h = stage_alloc(ctx, o_w + sw);
  std::memcpy(h, p.data(), sp);
  std::memcpy(h + o_w, work.data(), sw);
  char* dev = (char*)stage_launch(ctx, h, o_w + sw);
  ApplyProb* d = (ApplyProb*)dev;
  int32_t* w = (int32_t*)(dev + o_w);
  LaunchTimer lt(ctx, KK_OTHER, flops, bytes);
  k_apply(d, w, (int)(work.size() / 2), lds_for(lds), ctx->stream);
  p.clear();
}

void FillBatch::run(h2_ctx* ctx) {
  if (items.empty()) return;
  double bytes = 0;
  for (const FillItem& f : items) bytes += 8.0 * f.rows * f.cols;
  FillItem* d = upload_launch(ctx, items);
  LaunchTimer lt(ctx, KK_OTHER, 0.0, bytes);
  k_fill(d, (int)items.size(), ctx->stream);
  items.clear();
}

void TsqrBatch::add(const void* A, int64_t lda, int N, int m, bool transA, double* R, int64_t ldr,
                    int prec, const int32_t* col_off) {
  if (m <= 0) return;
  TsqrProb t{};
  t.A = A;
  t.lda = std::max<int64_t>(lda, 1);
  t.N = N;
  t.m = m;
  t.transA = transA ? 1 : 0;
  t.R = R;
  t.ldr = std::max<int64_t>(ldr, 1);
  t.prec = prec;
  t.col_off = col_off;
  p.push_back(t);
  max_m = std::max(max_m, m);
}

void TsqrBatch::run(h2_ctx* ctx) {
  if (p.empty()) return;
  // per problem: a register-blocked variant sized by m (the widest factored
  // width), else the streaming kernel in LDS, else the streaming kernel with
  // R in a global scratch slot and the row chunks in LDS (both in the slot
  // when even the chunks do not fit).
  // When the batch leaves most of the device idle, tall problems are cut into
  // row segments factored by separate workgroups, and a second launch
  // factors each stack of segment factors (a two-level TSQR tree; R agrees
  // with the one-level result up to the signs of its rows).
  const int lim = lds_limit_doubles();
  constexpr size_t kFillGroups = 1024;  // four workgroups per compute unit
  const size_t want = p.size() < kFillGroups ? kFillGroups / p.size() : 1;
  std::vector<std::pair<int, TsqrProb>> first, second;
  for (const TsqrProb& t : p) {
    const int v = tsqr_rb_variant(t.m, lim);
    int parts = 1;
    if (want > 1) {
      // segments of at least two row chunks of the variant (four times the
      // width for the streaming kernel), and taller than wide
      const int64_t seg_min = std::max<int64_t>(v ? 2 * tsqr_rb_chunk(v) : 4 * (int64_t)t.m, t.m + 1);
      parts = (int)std::min<int64_t>({(int64_t)want, t.N / seg_min, 16});
    }
    if (parts < 2) {
      first.push_back({v, t});
      continue;
    }
    // balanced segments of at least floor(N / parts) >= seg_min > m rows: the
    // factor of each fills all m rows of its slot in the stack (a factor of
    // fewer rows than m would leave rows of the slot unwritten)
    const int64_t ld_stack = (int64_t)parts * t.m;
    double* stack = ctx->ws.get<double>((size_t)ld_stack * t.m);
    const size_t es = t.prec ? sizeof(float) : sizeof(double);
    for (int q = 0; q < parts; ++q) {
      const int64_t r0 = (int64_t)t.N * q / parts, r1 = (int64_t)t.N * (q + 1) / parts;
      H2_REQUIRE(r1 - r0 >= t.m, H2_ERR_ARG, "tsqr: a row segment shorter than the width");
      TsqrProb u = t;
      u.A = (const char*)t.A + (size_t)(t.transA ? r0 * t.lda : r0) * es;
      u.N = (int32_t)(r1 - r0);
      u.R = stack + (size_t)q * t.m;
      u.ldr = ld_stack;
      first.push_back({v, u});
    }
    TsqrProb w{};
    w.A = stack;
    w.lda = ld_stack;
    w.N = (int32_t)ld_stack;
    w.m = t.m;
    w.transA = 0;
    w.prec = 0;
    w.col_off = nullptr;
    w.R = t.R;
    w.ldr = t.ldr;
    second.push_back({v, w});
  }
  WorkCounts wc = work_counts(ctx, (int)(first.size() + second.size()), KK_TSQR);
  if (wc.dev) {
    size_t i = 0;
    for (auto& e : first) e.second.work = wc.dev + i++;
    for (auto& e : second) e.second.work = wc.dev + i++;
  }
  auto launch = [&](const std::vector<std::pair<int, TsqrProb>>& list) {
    std::vector<TsqrProb> rb[4];
    size_t rb_need[4] = {0, 0, 0, 0};
    double rb_flops[4] = {0, 0, 0, 0}, rb_bytes[4] = {0, 0, 0, 0};
    size_t slot = 0, lds = 0;
    for (const auto& [v, t] : list) {
      double N = t.N, m = t.m, r = std::min(N, m);
      rb[v].push_back(t);
      rb_flops[v] += 2.0 * N * m * m - 2.0 * r * r * r / 3.0;
      rb_bytes[v] += 8.0 * (N * m + r * m);
      if (v) {
        rb_need[v] = std::max(rb_need[v], tsqr_rb_need(v, t.m));
      } else {
        size_t need = tsqr_lds_need(t.m, lim);
        if (need == 0) {  // R in a global scratch slot, the row chunks in LDS if they fit
          slot = std::max(slot, tsqr_scratch_need(t.m));
          lds = std::max(lds, tsqr_chunk_need(t.m, lim));
        } else {
          lds = std::max(lds, need);
        }
      }
    }
    for (int v = 1; v <= 3; ++v) {
      if (rb[v].empty()) continue;
      TsqrProb* d = upload_launch(ctx, rb[v]);
      LaunchTimer lt(ctx, KK_TSQR, wc.dev ? 0.0 : rb_flops[v], rb_bytes[v]);
      k_tsqr_rb(v, d, (int)rb[v].size(), rb_need[v], ctx->stream);
    }
    if (!rb[0].empty()) {
      double* scratch = slot ? ctx->ws.get<double>(slot * std::min<size_t>(rb[0].size(), 1024)) : nullptr;
      TsqrProb* d = upload_launch(ctx, rb[0]);
      LaunchTimer lt(ctx, KK_TSQR, wc.dev ? 0.0 : rb_flops[0], rb_bytes[0]);
      k_tsqr(d, (int)rb[0].size(), std::max<size_t>(lds, 1), slot, scratch, ctx->stream);
    }
  };
  launch(first);
  launch(second);
  if (wc.dev) {  // counts of all launches, resolved with the last one's timing
    dev_d2h(wc.host, wc.dev, sizeof(double) * wc.n, ctx->stream);
    if (!ctx->pending.empty()) {
      ctx->pending.back().work = wc.host;
      ctx->pending.back().nwork = wc.n;
    }
  }
  p.clear();
  max_m = 0;
}

void JacobiBatch::add(const double* R, int64_t ldr, int p_, int m, double* U, int64_t ldu,
                      double* sigma, int32_t* rank, double eps, double rtol, const int32_t* skip, int mode,
                      int rule) {
  H2_REQUIRE(m <= jacobi_max_len() && p_ <= jacobi_max_len(), H2_ERR_UNSUPPORTED,
             "jacobi: matrix larger than the kernels take");
  JacobiProb j{};
  j.R = R;
  j.ldr = std::max<int64_t>(ldr, 1);
  j.p = p_;
  j.m = m;
  j.U = U;
  j.ldu = std::max<int64_t>(ldu, 1);
  j.sigma = sigma;
  j.rank = rank;
  j.eps = eps;
  j.rtol = rtol;
  j.skip = skip;
  j.mode = mode;
  j.rule = rule;
  p.push_back(j);
  max_m = std::max(max_m, m);
}

void JacobiBatch::run(h2_ctx* ctx) {
  if (p.empty()) return;
  WorkCounts wc = work_counts(ctx, (int)p.size(), KK_JACOBI);
  if (wc.dev)
    for (size_t i = 0; i < p.size(); ++i) p[i].work = wc.dev + i;
  // small problems: one wavefront each; the rest: one workgroup each
  const size_t lim = (size_t)lds_limit_doubles();
  std::vector<JacobiProb> small, large;
  size_t per = 0, slot = 0, lds = 0;
  double flops_s = 0, bytes_s = 0, flops_l = 0, bytes_l = 0;
  for (const JacobiProb& j : p) {
    const size_t need = jacobi_need_doubles(j.p, j.m, j.mode);
    // one sweep over the pairs of players: 3 dot products and a rotation per pair
    const double pl = j.mode ? j.p : j.m, len = j.mode ? j.m : j.p;
    const double f = pl * (pl - 1) / 2 * (6.0 * len + (j.mode ? 0.0 : 6.0 * j.m));
    const double by = 8.0 * ((double)j.p * j.m + (j.U ? (double)j.m * j.m : 0.0));
    if (j.m <= jacobi_small_max_m() && j.p <= jacobi_small_max_m() && need <= lim) {
      small.push_back(j);
      per = std::max(per, need);
      flops_s += f;
      bytes_s += by;
    } else {
      large.push_back(j);
      if (need > lim)
        slot = std::max(slot, need);
      else
        lds = std::max(lds, need);
      flops_l += f;
      bytes_l += by;
    }
  }
  if (!small.empty()) {
    JacobiProb* d = upload_launch(ctx, small);
    LaunchTimer lt(ctx, KK_JACOBI, wc.dev ? 0.0 : flops_s, bytes_s);
    k_jacobi_small(d, (int)small.size(), (int)per, ctx->stream);
  }
  // the rest: medium problems on 256-thread groups, large ones on 1024
  std::vector<JacobiProb> grp[2];
  size_t gslot[2] = {0, 0}, glds[2] = {0, 0};
  for (const JacobiProb& j : large) {
    const int w = std::max(j.m, j.p) > jacobi_mid_max_m() ? 1 : 0;
    grp[w].push_back(j);
    const size_t need = jacobi_need_doubles(j.p, j.m, j.mode);
    if (need > lim)
      gslot[w] = std::max(gslot[w], need);
    else
      glds[w] = std::max(glds[w], need);
  }
  (void)slot;
  (void)lds;
  // a few medium problems beside wide ones join the wide launch: two launches
  // on the stream would run one after the other, each leaving most of the
  // device idle
  if (!grp[0].empty() && !grp[1].empty() && grp[0].size() < 128) {
    grp[1].insert(grp[1].end(), grp[0].begin(), grp[0].end());
    grp[0].clear();
    gslot[1] = std::max(gslot[1], gslot[0]);
    glds[1] = std::max(glds[1], glds[0]);
  }
  for (int w = 0; w < 2; ++w) {
    if (grp[w].empty()) continue;
    double* scratch = gslot[w] ? ctx->ws.get<double>(gslot[w] * std::min<size_t>(grp[w].size(), 1024)) : nullptr;
    JacobiProb* d = upload_launch(ctx, grp[w]);
    LaunchTimer lt(ctx, KK_JACOBI, wc.dev ? 0.0 : flops_l * grp[w].size() / large.size(), bytes_l * grp[w].size() / large.size());
    k_jacobi(d, (int)grp[w].size(), lds_for(glds[w]), gslot[w], scratch, w == 1, ctx->stream);
  }
  {  // relative-Frobenius ranks, from the singular values just written
    std::vector<JacobiProb> rel;
    for (const JacobiProb& j : p)
      if (j.rule == 1 && j.rank) rel.push_back(j);
    if (!rel.empty()) {
      JacobiProb* d = upload_launch(ctx, rel);
      LaunchTimer lt(ctx, KK_OTHER, 0.0, 8.0 * rel.size());
      k_rank_relf(d, (int)rel.size(), ctx->stream);
    }
  }
  if (wc.dev) {  // counts of both launches, resolved with the second one's timing
    dev_d2h(wc.host, wc.dev, sizeof(double) * wc.n, ctx->stream);
    if (!ctx->pending.empty()) {
      ctx->pending.back().work = wc.host;
      ctx->pending.back().nwork = wc.n;
    }
  }
  p.clear();
  max_m = 0;
}

std::vector<const double*> NormBatch::run(h2_ctx* ctx) {
  // pointer to sigma_max of every item (a zero for empty matrices)
  size_t n = items.size();
  std::vector<const double*> out(n);
  if (n == 0) return out;
  const double* zero = zeros(ctx, ctx->ws, 1);
  TsqrBatch ts;
  JacobiBatch jb;
  size_t rtot = 0, stot = 0;
  std::vector<size_t> roff(n), soff(n);
  for (size_t i = 0; i < n; ++i) {
    int mn = std::min(items[i].rows, items[i].cols);
    roff[i] = rtot;
    soff[i] = stot;
    rtot += (size_t)mn * mn;
    stot += mn;
  }
  double* R = ctx->ws.get<double>(std::max<size_t>(rtot, 1));
  double* S = ctx->ws.get<double>(std::max<size_t>(stot, 1));
  // g = min(rows, cols) <= norm2_max_dim(): the Gram / Lanczos kernel;
  // larger ones: R factor and the singular values of R
  std::vector<Norm2Prob> np;
  int gmax = 0;
  double nflops = 0, nbytes = 0;
  for (size_t i = 0; i < n; ++i) {
    const Item& it = items[i];
    int mn = std::min(it.rows, it.cols);
    if (mn == 0) {
      out[i] = zero;
      continue;
    }
    if (mn <= norm2_max_dim()) {
      np.push_back({it.A, std::max<int64_t>(it.lda, 1), it.rows, it.cols, S + soff[i]});
      out[i] = S + soff[i];
      gmax = std::max(gmax, mn);
      // Gram (upper triangle), Lanczos with two reorthogonalisations
      const double g = mn, s = std::max(it.rows, it.cols);
      nflops += s * g * (g + 1) + g * (2 * g * g + 4 * g * (g + 1));
      nbytes += 8.0 * it.rows * it.cols;
      continue;
    }
    // ||A||_2 = ||A^T||_2: factor the tall orientation
    bool tall = it.rows >= it.cols;
    ts.add(it.A, it.lda, std::max(it.rows, it.cols), mn, !tall, R + roff[i], mn);
    jb.add(R + roff[i], mn, mn, mn, nullptr, 1, S + soff[i], nullptr, 0.0);
    out[i] = S + soff[i];
  }
  if (!np.empty()) {
    Norm2Prob* d = upload_launch(ctx, np);
    LaunchTimer lt(ctx, KK_OTHER, nflops, nbytes);
    int ns_max = 0;
    for (const Norm2Prob& q : np) ns_max = std::max(ns_max, std::max(q.rows, q.cols));
    // samples staged per step: enough for the longest side, but no more
    // than the Lanczos vectors' space (g^2) holds, which keeps LDS per
    // problem, and so the problems resident per compute unit, at g^2 size
    int chunk = ns_max <= 16 ? 16 : ns_max <= 32 ? 32 : 64;
    while (chunk > 16 && chunk * gmax > gmax * gmax) chunk >>= 1;
    k_norm2(d, (int)np.size(), (int)norm2_need_doubles(gmax, chunk), chunk, ctx->stream);
  }
  ts.run(ctx);
  jb.run(ctx);
  if (!group.empty() && drop_rtol > 0.0) {
    H2_REQUIRE(group.size() == n, H2_ERR_ARG, "NormBatch: a group for every item or none");
    std::vector<int32_t> gptr(1, 0);
    for (size_t i = 0; i < n; ++i) {
      H2_REQUIRE(group[i] == (int32_t)gptr.size() - 1 || group[i] == (int32_t)gptr.size(), H2_ERR_ARG,
                 "NormBatch: groups must be numbered in item order");
      if (group[i] == (int32_t)gptr.size()) gptr.push_back((int32_t)i);
    }
    gptr.push_back((int32_t)n);
    std::vector<double*> vals(n);
    for (size_t i = 0; i < n; ++i) vals[i] = const_cast<double*>(out[i]);
    k_drop_small(upload_launch(ctx, vals), upload_launch(ctx, gptr), (int)gptr.size() - 1, drop_rtol, ctx->stream);
  }
  return out;
}

}  // namespace h2

h2_ctx::~h2_ctx() {
  for (h2_ctx* l : lanes) delete l;
  delete aux;
  for (auto& p : pending) {
    h2::dev_event_destroy(p.a);
    h2::dev_event_destroy(p.b);
  }
  for (void* e : ev_pool) h2::dev_event_destroy(e);
  h2::dev_event_destroy(drain);
  ws.release();
  for (auto& c : returned) h2::ctx_free(this, c.first);
  returned.clear();
  for (auto& c : cache) h2::ctx_free(this, c.first);
  cache.clear();
  for (auto& c : pool) h2::ctx_free(this, c.first);
  pool.clear();
  if (stage) h2::dev_free_host(stage);
  for (auto& c : prof_host) h2::dev_free_host(c.first);
  for (void* e : events) h2::dev_event_destroy(e);
  if (own_stream) h2::dev_stream_destroy(stream);
}
