// Phase 1: compressed induced cluster bases and the intermediate product G.
//
// Section 4 of the paper, for the row basis of X Y and (on the adjoint pair
// Y*, X*) for its column basis:
//   set-up   basis weights R_{Y,r} (Figure "basis_weights"), cluster basis
//            products P_{XY,s} = W_{X,s}^* V_{Y,s}, total weights Z_s
//            (Figure "total_weights") with the block scaling of Section 5;
//   sweep    Figure "induced_basis" level by level from the leaves: the
//            range of V_X (or Vhat_X) is kept by a Householder QR, the
//            remainder is truncated by an SVD at eps, transfer matrices are
//            cut from Qhat_t, and A_{t,s} = Q_t^* X|_{t x s} V_{Y,s} is kept.
// Every cluster of a level is processed by one batched launch per step; the
// ranks chosen on a level are read back once before the next level.
//
// G is then formed on the product block tree T^XY: every terminated triple
// (t,s,r) contributes P_row X|_{ts} Y|_{sr} P_col in the coefficients of the
// new bases (projection only on a subdivided or inadmissible factor side),
// contributions are pushed to the leaves of T^XY with the new transfer
// matrices, and inadmissible leaves are expanded to dense blocks together
// with the products of two nearfield blocks.
#include <cmath>

#include <algorithm>
#include <array>
#include <condition_variable>
#include <exception>
#include <mutex>
#include <thread>

#include "internal.h"

namespace h2 {

struct P1Side {
  Basis Q;                                   // new isometric nested basis
  std::vector<int32_t> k1;                   // rank of the kept V_X part
  std::vector<double*> RXP;                  // [R_{X,t}; 0], k_t x k, ld k_t
  std::vector<double*> A;                    // A_{t,s} for s in C_t: k_t x (k |C_t|), ld k_t
  std::vector<int32_t> cpos;                 // per stored block of X': position in C_{t}
  std::vector<double*> P;                    // P_{XY,s}, k x k
};

// Completion of the levels of the two induced-basis passes (both run from
// the leaves up), for the parts of G that need the bases of one level only.
// A pass records an event on its stream after a level and publishes the
// level; a waiter orders its own stream after both events.
struct LevelSignal {
  std::mutex mu;
  std::condition_variable cv;
  int low[2];                // lowest level finished by each pass (depth + 1: none yet)
  bool stop = false;         // set when a pass ends early (an error)
  std::vector<void*> ev[2];  // per pass and level
  explicit LevelSignal(int depth) {
    for (int s = 0; s < 2; ++s) {
      low[s] = depth + 1;
      ev[s].assign(depth + 1, nullptr);
      for (auto& e : ev[s]) e = dev_event_create();
    }
  }
  ~LevelSignal() {
    for (auto& v : ev)
      for (void* e : v) dev_event_destroy(e);
  }
  void done(int side, int l, void* stream) {
    dev_event_record(ev[side][l], stream);
    {
      std::lock_guard<std::mutex> lk(mu);
      low[side] = l;
    }
    cv.notify_all();
  }
  // true once both passes have finished level l; false if stopped before
  bool wait(int l) {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return (low[0] <= l && low[1] <= l) || stop; });
    return low[0] <= l && low[1] <= l;
  }
  void abort() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
    }
    cv.notify_all();
  }
};

static int uniform_rank(const Basis& B) {
  int k = B.rank.empty() ? 0 : B.rank[0];
  for (int r : B.rank) H2_REQUIRE(r == k, H2_ERR_UNSUPPORTED, "input bases must have one rank");
  return k;
}

// One pass of Figure "induced_basis" for the product X Y given as views.
static void induced_pass(h2_ctx* ctx, const View& X, const View& Y, double eps, Arena& keep,
                         P1Side& out, int step_setup, int step_sweep, LevelSignal* lsig, int side) {
  const TreeH& T = *X.m->ct;
  const int ncl = T.ncl, D = T.depth;
  const int k = uniform_rank(X.rowb());
  H2_REQUIRE(uniform_rank(Y.rowb()) == k && uniform_rank(X.colb()) == k && uniform_rank(Y.colb()) == k,
             H2_ERR_UNSUPPORTED, "X and Y must have the same rank");
  const Basis& VX = X.rowb();
  const Basis& WX = X.colb();
  const Basis& VY = Y.rowb();
  const Basis& WY = Y.colb();
  Arena& ws = ctx->ws;
  GemmBatch g;
  g.prec = ctx->prec;
  step_begin(ctx, step_setup);

  // ---- basis weights of W_Y (bottom-up thin QR) ----
  std::vector<double*> RY(ncl);
  std::vector<int> lY(ncl);
  for (int c = 0; c < ncl; ++c) RY[c] = ws.get<double>((size_t)k * k);  // rows < lY[c] are written
  {
    TsqrBatch ts;
    for (int c = T.first(D); c < ncl; ++c) {
      lY[c] = (int)std::min<int64_t>(k, T.size[c]);
      ts.add(WY.leaf[c], WY.leaf_ld[c], (int)T.size[c], k, false, RY[c], k);
    }
    ts.run(ctx);
    for (int l = D - 1; l >= 0; --l) {
      for (int c = T.first(l); c < T.first(l + 1); ++c) {
        int c1 = 2 * c + 1, c2 = 2 * c + 2;
        int rows = lY[c1] + lY[c2];
        double* Wh = ws.get<double>((size_t)std::max(rows, 1) * k);
        g.out(Wh, rows, lY[c1], k);
        g.term(RY[c1], k, false, WY.tr[c1], WY.tr_ld[c1], false, k);
        g.out(Wh + lY[c1], rows, lY[c2], k);
        g.term(RY[c2], k, false, WY.tr[c2], WY.tr_ld[c2], false, k);
        lY[c] = std::min(k, rows);
        ts.add(Wh, rows, rows, k, false, RY[c], k);
      }
      g.run(ctx);
      ts.run(ctx);
    }
  }
  // ---- cluster basis products P_s = W_{X,s}^* V_{Y,s} ----
  out.P.assign(ncl, nullptr);
  for (int c = 0; c < ncl; ++c) out.P[c] = ws.get<double>((size_t)k * k);
  for (int c = T.first(D); c < ncl; ++c) {
    g.out(out.P[c], k, k, k);
    g.term(WX.leaf[c], WX.leaf_ld[c], true, VY.leaf[c], VY.leaf_ld[c], false, (int)T.size[c]);
  }
  g.run(ctx);
  std::vector<double*> PE(ncl, nullptr);  // P_s E_{Y,s}
  for (int l = D; l >= 1; --l) {
    for (int c = T.first(l); c < T.first(l + 1); ++c) {
      PE[c] = ws.get<double>((size_t)k * k);
      g.out(PE[c], k, k, k);
      g.term(out.P[c], k, false, VY.tr[c], VY.tr_ld[c], false, k);
    }
    g.run(ctx);
    for (int c = T.first(l - 1); c < T.first(l); ++c) {
      g.out(out.P[c], k, k, k);
      for (int q = 1; q <= 2; ++q)
        g.term(WX.tr[2 * c + q], WX.tr_ld[2 * c + q], true, PE[2 * c + q], k, false, k);
    }
    g.run(ctx);
  }
  // ---- total weights of (V_Y, Y), top-down, blocks scaled by 1/||S R^*||_2 ----
  const BlockTreeH& BY = Y.bt();
  std::vector<double*> M(BY.nblocks(), nullptr);
  NormBatch nb;
  nb.drop_rtol = kBlockRtol;  // per level of the block tree (blocks are stored level by level)
  std::vector<int> nbi(BY.nblocks(), -1);
  int cur_lvl = -1, gid = -1;
  for (int b = 0; b < BY.nblocks(); ++b) {
    if (Y.type(b) != BT_ADM) continue;
    int r = Y.vcol(b);
    M[b] = ws.get<double>((size_t)k * k);
    g.out(M[b], std::max(lY[r], 1), lY[r], k);
    g.term(RY[r], k, false, Y.ptr(b), Y.ld(b), !Y.T, k);  // R_{Y,r} S_{Y,sr}^*
    nbi[b] = (int)nb.items.size();
    const int lv = TreeH::level(Y.vrow(b));
    if (lv != cur_lvl) {
      cur_lvl = lv;
      ++gid;
    }
    nb.add(M[b], std::max(lY[r], 1), lY[r], k, gid);
  }
  g.run(ctx);
  std::vector<const double*> sig = nb.run(ctx);
  std::vector<double*> Z(ncl, nullptr);
  std::vector<int> zr(ncl, 0);
  ScopedArena lvl(ctx);  // per-level temporaries
  for (int l = 0; l <= D; ++l) {
    lvl.reset();
    // the stacked weights in runs of at most run_scratch bytes, each reduced
    // to its R factors before the run's memory is reused
    TsqrBatch ts;
    size_t pend = 0;
    auto flush = [&] {
      g.run(ctx);
      ts.run(ctx);
      lvl.reset();
      pend = 0;
    };
    for (int s = T.first(l); s < T.first(l + 1); ++s) {
      const int32_t* bl;
      int cnt;
      Y.row_blocks(s, bl, cnt);
      int N = l > 0 ? zr[TreeH::parent(s)] : 0;
      for (int q = 0; q < cnt; ++q)
        if (Y.type(bl[q]) == BT_ADM) N += lY[Y.vcol(bl[q])];
      Z[s] = ws.get<double>((size_t)k * k);
      zr[s] = std::min(N, k);
      if (N == 0) continue;
      const size_t e = 8 * (size_t)N * k;
      if (pend > 0 && pend + e > ctx->run_scratch) flush();
      double* Gh = lvl.get<double>((size_t)N * k);
      pend += e;
      int row = 0;
      if (l > 0 && zr[TreeH::parent(s)] > 0) {
        int zp = zr[TreeH::parent(s)];
        g.out(Gh, N, zp, k);
        g.term(Z[TreeH::parent(s)], k, false, VY.tr[s], VY.tr_ld[s], true, k);
        row += zp;
      }
      for (int q = 0; q < cnt; ++q) {
        int b = bl[q];
        if (Y.type(b) != BT_ADM) continue;
        int lr = lY[Y.vcol(b)];
        g.out(Gh + row, N, lr, k);
        g.copy(M[b], std::max(lr, 1), false, k, 1.0, sig[nbi[b]], 2);
        row += lr;
      }
      ts.add(Gh, N, N, k, false, Z[s], k);
    }
    flush();
  }
  // S_{X,t's'} P_{s'} E_{Y,s'} for admissible blocks of X below the root
  const BlockTreeH& BX = X.bt();
  std::vector<double*> SPE(BX.nblocks(), nullptr);
  for (int b = 0; b < BX.nblocks(); ++b) {
    if (X.type(b) != BT_ADM || X.vrow(b) == 0) continue;
    SPE[b] = ws.get<double>((size_t)k * k);
    g.out(SPE[b], k, k, k);
    g.term(X.ptr(b), X.ld(b), X.T, PE[X.vcol(b)], k, false, k);
  }
  g.run(ctx);
  step_end(ctx, step_setup);

  // ---- the sweep of Figure "induced_basis" ----
  step_begin(ctx, step_sweep);
  out.Q.resize(ncl);
  out.k1.assign(ncl, 0);
  out.RXP.assign(ncl, nullptr);
  out.A.assign(ncl, nullptr);
  out.cpos.assign(BX.nblocks(), -1);
  std::vector<std::vector<int32_t>> Cb(ncl);  // blocks (t, s), s in C_t, sorted by s
  for (int t = 0; t < ncl; ++t) {
    const int32_t* bl;
    int cnt;
    X.row_blocks(t, bl, cnt);
    for (int q = 0; q < cnt; ++q)
      if (X.type(bl[q]) != BT_ADM) {
        out.cpos[bl[q]] = (int32_t)Cb[t].size();
        Cb[t].push_back(bl[q]);
      }
  }
  for (int l = D; l >= 0; --l) {
    lvl.reset();  // B_t, V_X and the scaled remainder of one level at a time
    const int c0 = T.first(l), c1 = T.first(l + 1), nc = c1 - c0;
    const bool leaf = l == D;
    std::vector<int> rows(nc), ncols(nc), kk1(nc);
    std::vector<double*> Bt(nc), Vr(nc), VXw(nc);
    std::vector<std::vector<int>> offs(nc);
    // (a) the blocks X|_{t x s} V_{Y,s} (leaf) or Ahat_{t,s} (non-leaf), the V_X part
    for (int i = 0; i < nc; ++i) {
      int t = c0 + i;
      int m = leaf ? (int)T.size[t] : out.Q.rank[2 * t + 1] + out.Q.rank[2 * t + 2];
      rows[i] = m;
      int nC = (int)Cb[t].size();
      Bt[i] = lvl.get<double>((size_t)std::max(m, 1) * k * std::max(nC, 1));
      VXw[i] = lvl.get<double>((size_t)std::max(m, 1) * k);
      if (leaf) {
        for (int j = 0; j < nC; ++j) {
          int b = Cb[t][j], s = X.vcol(b);
          g.out(Bt[i] + (size_t)j * k * m, m, m, k);
          g.term(X.ptr(b), X.ld(b), X.T, VY.leaf[s], VY.leaf_ld[s], false, (int)T.size[s]);
        }
        g.out(VXw[i], m, m, k);
        g.copy(VX.leaf[t], VX.leaf_ld[t], false, k);
      } else {
        int o = 0;
        offs[i].clear();
        for (int q = 1; q <= 2; ++q) {
          int ch = 2 * t + q;
          offs[i].push_back(o);
          g.out(VXw[i] + o, m, out.Q.rank[ch], k);
          g.term(out.RXP[ch], std::max(out.Q.rank[ch], 1), false, VX.tr[ch], VX.tr_ld[ch], false, k);
          o += out.Q.rank[ch];
        }
        for (int j = 0; j < nC; ++j) {
          int s = X.vcol(Cb[t][j]);
          for (int q = 1; q <= 2; ++q) {
            int ch = 2 * t + q, kc = out.Q.rank[ch];
            g.out(Bt[i] + (size_t)j * k * m + offs[i][q - 1], m, kc, k);
            for (int p2 = 1; p2 <= 2; ++p2) {
              int sc = 2 * s + p2;
              int bc = X.find(ch, sc);
              H2_REQUIRE(bc >= 0, H2_ERR_SHAPE, "missing child block");
              if (X.type(bc) == BT_ADM)
                g.term(out.RXP[ch], std::max(kc, 1), false, SPE[bc], k, false, k);
              else
                g.term(out.A[ch] + (size_t)out.cpos[bc] * k * kc, std::max(kc, 1), false, VY.tr[sc],
                       VY.tr_ld[sc], false, k);
            }
          }
        }
      }
    }
    g.run(ctx);
    // (b) block norms (Section 5); blocks at most kBlockRtol of the level's
    //     largest are zero up to rounding and are dropped
    NormBatch nrm;
    nrm.drop_rtol = kBlockRtol;
    std::vector<std::vector<int>> ni(nc);
    for (int i = 0; i < nc; ++i) {
      int t = c0 + i;
      for (size_t j = 0; j < Cb[t].size(); ++j) {
        ni[i].push_back((int)nrm.items.size());
        nrm.add(Bt[i] + j * k * rows[i], std::max(rows[i], 1), rows[i], k, 0);
      }
    }
    std::vector<const double*> ns = nrm.run(ctx);
    // (c) scaled remainder blocks X V_Y Z_s^* / ||.||
    for (int i = 0; i < nc; ++i) {
      int t = c0 + i, m = rows[i];
      int nco = 0;
      for (int b : Cb[t]) nco += zr[X.vcol(b)];
      ncols[i] = nco;
      Vr[i] = lvl.get<double>((size_t)m * std::max(nco, 1));
      int col = 0;
      for (size_t j = 0; j < Cb[t].size(); ++j) {
        int s = X.vcol(Cb[t][j]);
        if (zr[s] == 0) continue;
        g.out(Vr[i] + (size_t)col * m, m, m, zr[s]);
        g.term(Bt[i] + j * k * m, m, false, Z[s], k, true, k, 1.0, ns[ni[i][j]], 2);
        col += zr[s];
      }
    }
    g.run(ctx);
    // (d) the range of V_X kept, the remainder truncated at eps (SVD of V_X
    //     from its R factor, Householder QR of V_X V', SVD of the rest)
    std::vector<KeptItem> kit(nc);
    for (int i = 0; i < nc; ++i) kit[i] = {rows[i], VXw[i], rows[i], k, Vr[i], rows[i], ncols[i]};
    KeptOut ko;
    kept_compress(ctx, kit, level_eps(ctx, eps, D, l), keep, ko);
    // (e) Q_t, transfers, A_{t,s} = Q_t^* (...), [R_X; 0]
    std::vector<double*> Qn(nc);
    for (int i = 0; i < nc; ++i) {
      int t = c0 + i;
      kk1[i] = ko.k1[i];
      int kt = ko.k1[i] + ko.k2[i];
      H2_REQUIRE(kt >= 1, H2_ERR_NUMERIC, "phase 1: empty cluster basis");
      out.Q.rank[t] = kt;
      out.k1[t] = kk1[i];
      Qn[i] = ko.Q[i];
    }
    for (int i = 0; i < nc; ++i) {
      int t = c0 + i, m = rows[i], kt = out.Q.rank[t];
      if (leaf) {
        out.Q.leaf[t] = Qn[i];
        out.Q.leaf_ld[t] = m;
      } else {
        for (int q = 1; q <= 2; ++q) {
          out.Q.tr[2 * t + q] = Qn[i] + offs[i][q - 1];
          out.Q.tr_ld[2 * t + q] = m;
        }
      }
      int nC = (int)Cb[t].size();
      out.A[t] = ws.get<double>((size_t)kt * k * std::max(nC, 1));
      if (nC > 0) {
        g.out(out.A[t], kt, kt, k * nC);
        g.term(Qn[i], m, true, Bt[i], m, false, m);
      }
      out.RXP[t] = ko.RKP[i];
    }
    g.run(ctx);
    if (lsig) lsig->done(side, l, ctx->stream);
  }
  step_end(ctx, step_sweep);
}

void phase1(h2_ctx* ctx, const h2_matrix* Xm, const h2_matrix* Ym, double eps, int prec,
            h2_product* G) {
  const TreeH& T = *Xm->c.ct;
  H2_REQUIRE(T.same_as(*Ym->c.ct), H2_ERR_SHAPE, "X and Y must share the cluster tree");
  ctx->prec = prec;
  G->ctx = ctx;
  G->mem.bind(ctx);
  View X{&Xm->c, false}, Y{&Ym->c, false};
  View Yt{&Ym->c, true}, Xt{&Xm->c, true};
  const BlockTreeH& BX = *Xm->c.bt;
  const BlockTreeH& BY = *Ym->c.bt;
  const int nbx = BX.nblocks(), nby = BY.nblocks();
  // operand tables of the factor blocks of a triple: X's and Y's blocks
  std::vector<const double*> tX(nbx), tY(nby);
  std::vector<int64_t> lX(nbx), lY(nby);
  for (int b = 0; b < nbx; ++b) {
    tX[b] = Xm->c.blk[b];
    lX[b] = Xm->c.ld_of(b);
  }
  for (int b = 0; b < nby; ++b) {
    tY[b] = Ym->c.blk[b];
    lY[b] = Ym->c.ld_of(b);
  }
  // The dense leaf blocks of T^XY start with the sum of their nearfield-
  // times-nearfield triples and the product tree T^XY is symbolic (block
  // trees only); neither needs a basis, so both are done on a second
  // auxiliary context (host thread and stream) while the two induced-basis
  // passes run.  The dense blocks are the leaf pairs (t, r) joined by a
  // nearfield block (t, s) of X and (s, r) of Y (a block of T^XY is dense
  // exactly when such a triple ends in it); their products are launched
  // before the product tree is built (on a host thread of its own).  The
  // same context then forms the part of G that needs the bases of one level
  // only, level by level as the passes finish them.  The parents' share of
  // S and the projected part Q_t S Q^W_r^* of the dense blocks are added
  // after the passes.
  ProductTreeH PT;
  std::exception_ptr sym_err;
  struct Joiner {
    std::thread th;
    void join() {
      if (th.joinable()) th.join();
    }
    ~Joiner() { join(); }
  } sym;
  sym.th = std::thread([&] {  // host work only
    try {
      PT = build_product_tree(X, Y, T.ncl);
    } catch (...) {
      sym_err = std::current_exception();
    }
  });
  std::vector<std::vector<std::pair<int, double*>>> dn_of(T.ncl);  // leaf t: (r, block) by r
  auto dense_block = [&](int t, int r) {
    const auto& dl = dn_of[t];
    auto it = std::lower_bound(dl.begin(), dl.end(), std::make_pair(r, (double*)nullptr));
    H2_REQUIRE(it != dl.end() && it->first == r, H2_ERR_SHAPE, "dense leaf of T^XY without nearfield triple");
    return it->second;
  };
  h2_ctx* nf_ctx = aux_ctx(aux_ctx(ctx));
  G->mem_nf.bind(nf_ctx);
  const int k = uniform_rank(Xm->c.V);
  P1Side row, col;
  LevelSignal sig(T.depth);
  // S (kt x kr) of every block of T^XY, in the coefficients of the new bases
  std::vector<double*> S;
  AuxRun nfrun(ctx, nf_ctx, [&](h2_ctx* a) {
    step_begin(a, 1);
    std::vector<int32_t> sizes(T.ncl);
    int64_t leaf_max = 0;
    for (int c = 0; c < T.ncl; ++c) {
      sizes[c] = (int32_t)T.size[c];
      if (T.leaf(c)) leaf_max = std::max(leaf_max, T.size[c]);
    }
    TriBatch tnn;
    tnn.prec = prec;
    tnn.block = true;  // 64 x 64 parts of the dense products, one workgroup each
    std::vector<Triple> nn;
    std::vector<std::array<int32_t, 4>> rowl;  // (r, s, bx, by) of one leaf t
    double f_nn = 0;
    for (int t = T.first(T.depth); t < T.ncl; ++t) {
      rowl.clear();
      const int32_t* bl;
      int cnt;
      X.row_blocks(t, bl, cnt);
      for (int q = 0; q < cnt; ++q) {
        if (X.type(bl[q]) != BT_INADM) continue;
        const int sm = X.vcol(bl[q]);
        const int32_t* bl2;
        int cnt2;
        Y.row_blocks(sm, bl2, cnt2);
        for (int q2 = 0; q2 < cnt2; ++q2)
          if (Y.type(bl2[q2]) == BT_INADM) rowl.push_back({Y.vcol(bl2[q2]), sm, bl[q], bl2[q2]});
      }
      std::sort(rowl.begin(), rowl.end());
      for (size_t i = 0; i < rowl.size();) {
        const int r = rowl[i][0];
        const int q0 = (int)nn.size();
        for (; i < rowl.size() && rowl[i][0] == r; ++i) {
          nn.push_back({rowl[i][1], rowl[i][2], rowl[i][3], TK_NN});
          f_nn += 2.0 * T.size[t] * T.size[r] * T.size[rowl[i][1]];
        }
        double* D = G->mem_nf.get<double>((size_t)T.size[t] * T.size[r]);
        dn_of[t].push_back({r, D});
        tnn.out(D, T.size[t], (int)T.size[t], (int)T.size[r], q0, (int)nn.size(), false);
      }
    }
    // operand tables indexed by the factor blocks of a triple
    const double* const* d_tX = upload(a, tX);
    const int64_t* d_lX = upload(a, lX);
    const double* const* d_tY = upload(a, tY);
    const int64_t* d_lY = upload(a, lY);
    auto family = [&](const int32_t* tri, const double* const* A, const int64_t* la, const double* const* Bt,
                      const int64_t* lb, int kind, bool tB, const int32_t* ks) {
      TriFamily f{};
      f.tri = tri;
      f.A = A;
      f.lda = la;
      f.B = Bt;
      f.ldb = lb;
      f.ks = ks;
      f.k = k;
      f.kind = kind;
      f.tA = 0;
      f.tB = tB ? 1 : 0;
      return f;
    };
    // N_X N_Y over the leaf size of the middle cluster
    tnn.fam = family((const int32_t*)upload(a, nn.empty() ? std::vector<Triple>{{0, 0, 0, -1}} : nn), d_tX, d_lX,
                     d_tY, d_lY, TK_NN, false, upload(a, sizes));
    sym.join();
    if (sym_err) std::rethrow_exception(sym_err);
    const int32_t* d_tri = PT.tri.empty() ? (const int32_t*)upload(a, std::vector<Triple>{{0, 0, 0, -1}})
                                          : (const int32_t*)upload(a, PT.tri);
    // The dense products fill the whole device; launched while the passes
    // still factorize the wide lower levels they would hold those launches
    // back.  They start once both passes are three levels from the leaves,
    // where the passes' launches leave most compute units idle.
    H2_REQUIRE(sig.wait(std::max(0, T.depth - 3)), H2_ERR_DEVICE, "phase 1: a basis pass stopped early");
    tnn.run(a, f_nn);
    step_end(a, 1);

    // ---- G, the part of each level that needs the bases of that level only ----
    // Sloc_b = TNA_b R^c_r^* + R_t Mm_b with TNA_b the sum of A_{t,s} S_Y over
    // the NA triples and Mm_b = (sum of S_X P S_Y over AA triples) R^c_r^* +
    // sum of S_X A^c^* over AN triples; it is formed for each level of T^XY as
    // soon as both passes have finished that level.  The projections of the
    // parents' S are added top-down once the passes are done.
    step_begin(a, 4);
    const BlockTreeH& B = *PT.bt;
    Arena& ws = a->ws;
    GemmBatch g;
    g.prec = prec;
    S.assign(B.nblocks(), nullptr);
    auto cnt = [&](int b, int kind) { return PT.kind_cnt[4 * (size_t)b + kind]; };
    std::vector<const double*> tPS(nby, nullptr), tAr(nbx, nullptr), tAc(nby, nullptr);
    std::vector<int64_t> lPS(nby, k), lAr(nbx, 1), lAc(nby, 1);
    TriFamily fAA{};
    ScopedArena tmp(a);  // the triple sums of one run of blocks at a time
    // blocks [c0b, c1b) of one level whose ranks exceed the fused kernel's:
    // the three triple sums, then S_b = TNA_b R^c_r^* + R_t Mm_b
    auto unfused_run = [&](int c0b, int c1b, const TriFamily& fNA, const TriFamily& fAN) {
      tmp.reset();
      TriBatch taa, tna, tan_;
      taa.fam = fAA;
      tna.fam = fNA;
      tan_.fam = fAN;
      taa.prec = tna.prec = tan_.prec = prec;
      taa.block = tna.block = true;  // untransposed operands: 64 x 64 parts on the block kernel
      const int nb = c1b - c0b;
      std::vector<double*> TAA(nb, nullptr), TNA(nb, nullptr), Mm(nb, nullptr);
      double f_aa = 0, f_na = 0, f_an = 0;
      for (int b = c0b; b < c1b; ++b) {
        const int i = b - c0b, kt = row.Q.rank[B.t[b]];
        if (cnt(b, TK_AA)) {
          TAA[i] = tmp.get<double>((size_t)k * k);
          taa.out(TAA[i], k, k, k, PT.tri_ptr[b], PT.tri_ptr[b + 1]);
          f_aa += 2.0 * k * k * k * cnt(b, TK_AA);
        }
        if (cnt(b, TK_NA) && kt > 0) {
          TNA[i] = tmp.get<double>((size_t)kt * k);
          tna.out(TNA[i], kt, kt, k, PT.tri_ptr[b], PT.tri_ptr[b + 1]);
          f_na += 2.0 * kt * k * k * cnt(b, TK_NA);
        }
      }
      taa.run(a, f_aa);
      tna.run(a, f_na);
      for (int b = c0b; b < c1b; ++b) {
        const int i = b - c0b, r = B.s[b], kr = col.Q.rank[r];
        if ((cnt(b, TK_AN) || TAA[i]) && kr > 0) {
          Mm[i] = tmp.get<double>((size_t)k * kr);
          g.out(Mm[i], k, k, kr);
          if (TAA[i]) g.term(TAA[i], k, false, col.RXP[r], kr, true, k);
          if (cnt(b, TK_AN)) {
            tan_.out(Mm[i], k, k, kr, PT.tri_ptr[b], PT.tri_ptr[b + 1], TAA[i] != nullptr);
            f_an += 2.0 * k * k * kr * cnt(b, TK_AN);
          }
        }
      }
      g.run(a);  // TAA R^c^* first (overwrites), then the AN triples accumulate
      tan_.run(a, f_an);
      // dense leaves (S[b] null) keep their coupling in the run's scratch
      // and add Q_t S Q^W_r^* to their block at once
      std::vector<double*> Sd(nb, nullptr), QS(nb, nullptr);
      for (int b = c0b; b < c1b; ++b) {
        const int i = b - c0b, t = B.t[b], r = B.s[b], kt = row.Q.rank[t], kr = col.Q.rank[r];
        double* Sb = S[b] ? S[b] : (Sd[i] = tmp.get<double>((size_t)std::max(kt, 1) * std::max(kr, 1)));
        g.out(Sb, std::max(kt, 1), kt, kr);  // zero without terms
        if (TNA[i]) g.term(TNA[i], kt, false, col.RXP[r], std::max(kr, 1), true, k);
        if (Mm[i]) g.term(row.RXP[t], std::max(kt, 1), false, Mm[i], k, false, k);
      }
      g.run(a);
      for (int b = c0b; b < c1b; ++b) {
        const int i = b - c0b, t = B.t[b], r = B.s[b], kt = row.Q.rank[t], kr = col.Q.rank[r];
        if (!Sd[i] || kt == 0 || kr == 0) continue;
        const int mt = (int)T.size[t];
        QS[i] = tmp.get<double>((size_t)mt * kr);
        g.out(QS[i], mt, mt, kr);
        g.term(row.Q.leaf[t], row.Q.leaf_ld[t], false, Sd[i], kt, false, kt);
      }
      g.run(a);
      for (int b = c0b; b < c1b; ++b) {
        const int i = b - c0b, t = B.t[b], r = B.s[b], kr = col.Q.rank[r];
        if (!QS[i]) continue;
        const int mt = (int)T.size[t], nr = (int)T.size[r];
        g.out(dense_block(t, r), mt, mt, nr, true);
        g.term(QS[i], mt, false, col.Q.leaf[r], col.Q.leaf_ld[r], true, kr);
      }
      g.run(a);
    };
    const int32_t* d_bt = nullptr;    // (t, r) per block of T^XY, for the fused launches
    const int32_t* d_tptr = nullptr;  // triple ranges per block of T^XY
    for (int l = T.depth; l >= 0; --l) {
      H2_REQUIRE(sig.wait(l), H2_ERR_DEVICE, "phase 1: a basis pass stopped early");
      dev_stream_wait(a->stream, sig.ev[0][l]);
      dev_stream_wait(a->stream, sig.ev[1][l]);
      if (l == T.depth) {  // P_{XY,s} S_{Y,sr} for admissible blocks of Y (P from the row set-up)
        for (int b = 0; b < nby; ++b) {
          if (BY.type[b] != BT_ADM) continue;
          double* ps = ws.get<double>((size_t)k * k);
          tPS[b] = ps;
          g.out(ps, k, k, k);
          g.term(row.P[BY.t[b]], k, false, Ym->c.blk[b], Ym->c.ld_of(b), false, k);
        }
        g.run(a);
        fAA = family(d_tri, d_tX, d_lX, upload(a, tPS), upload(a, lPS), TK_AA, false, nullptr);  // S_X (P S_Y)
      }
      // A_{t,s} of the blocks of X and A^c of the blocks of Y on this level
      for (int b = BX.lvl[l]; b < BX.lvl[l + 1]; ++b)
        if (BX.type[b] != BT_ADM && row.cpos[b] >= 0) {
          const int kt = row.Q.rank[X.vrow(b)];
          tAr[b] = row.A[X.vrow(b)] + (size_t)row.cpos[b] * k * kt;
          lAr[b] = std::max(kt, 1);
        }
      for (int b = BY.lvl[l]; b < BY.lvl[l + 1]; ++b)
        if (BY.type[b] != BT_ADM && col.cpos[b] >= 0) {
          const int r = BY.s[b], kr = col.Q.rank[r];
          tAc[b] = col.A[r] + (size_t)col.cpos[b] * k * kr;
          lAc[b] = std::max(kr, 1);
        }
      const int b0 = B.lvl[l], b1 = B.lvl[l + 1];
      if (b1 == b0) continue;
      int ktmax = 0, krmax = 0;
      for (int c = T.first(l); c < T.first(l + 1); ++c) {
        ktmax = std::max(ktmax, row.Q.rank[c]);
        krmax = std::max(krmax, col.Q.rank[c]);
      }
      if (k <= 64 && ktmax <= 64 && krmax <= 64) {
        // one fused launch: the three triple sums and both closing products
        if (!d_bt) {
          std::vector<int32_t> bt(2 * (size_t)B.nblocks());
          for (int b = 0; b < B.nblocks(); ++b) {
            bt[2 * (size_t)b] = B.t[b];
            bt[2 * (size_t)b + 1] = B.s[b];
          }
          d_bt = upload(a, bt);
          d_tptr = upload(a, PT.tri_ptr);
        }
        const int c0 = T.first(l), nc = T.first(l + 1) - c0;
        const int bx0 = BX.lvl[l], nbxl = BX.lvl[l + 1] - bx0, by0 = BY.lvl[l], nbyl = BY.lvl[l + 1] - by0;
        const int nb = b1 - b0;
        size_t total = 0, total_adm = 0;
        double flops = 0, bytes = 0;
        for (int b = b0; b < b1; ++b) {
          const int kt = row.Q.rank[B.t[b]], kr = col.Q.rank[B.s[b]];
          const size_t e = (size_t)std::max(kt, 1) * std::max(kr, 1);
          total += e;
          if (B.type[b] == BT_ADM) total_adm += e;
          const double naa = cnt(b, TK_AA), nna = kt ? cnt(b, TK_NA) : 0, nan = kr ? cnt(b, TK_AN) : 0;
          flops += 2.0 * k * k * (k * naa + kt * nna + kr * nan) + 2.0 * kt * k * kr * ((nna > 0) + (naa + nan > 0)) +
                   (naa > 0 ? 2.0 * k * k * kr : 0.0);
          bytes += 8.0 * kt * kr;
        }
        // couplings of admissible blocks stay in G; the others (subdivided
        // blocks and dense leaves) are needed only until the top-down
        // projections below, and live in the workspace
        double* Sl = G->mem_nf.get<double>(std::max<size_t>(total_adm, 1));
        double* Sw = ws.get<double>(std::max<size_t>(total - total_adm, 1));
        // the level's tables, packed into one upload
        auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
        const size_t o_kc = al(4 * (size_t)nc), o_rr = o_kc + al(4 * (size_t)nc), o_rc = o_rr + al(8 * (size_t)nc),
                     o_s = o_rc + al(8 * (size_t)nc), o_ar = o_s + al(8 * (size_t)nb),
                     o_lar = o_ar + al(8 * (size_t)nbxl), o_ac = o_lar + al(8 * (size_t)nbxl),
                     o_lac = o_ac + al(8 * (size_t)nbyl), o_end = o_lac + al(8 * (size_t)nbyl);
        char* h = stage_alloc(a, o_end);
        int32_t* hkr = (int32_t*)h;
        int32_t* hkc = (int32_t*)(h + o_kc);
        const double** hrr = (const double**)(h + o_rr);
        const double** hrc = (const double**)(h + o_rc);
        double** hs = (double**)(h + o_s);
        for (int i = 0; i < nc; ++i) {
          hkr[i] = row.Q.rank[c0 + i];
          hkc[i] = col.Q.rank[c0 + i];
          hrr[i] = row.RXP[c0 + i];
          hrc[i] = col.RXP[c0 + i];
        }
        for (int b = b0, off = 0, offw = 0; b < b1; ++b) {
          const int kt = row.Q.rank[B.t[b]], kr = col.Q.rank[B.s[b]];
          const int e = std::max(kt, 1) * std::max(kr, 1);
          if (B.type[b] == BT_ADM) {
            S[b] = hs[b - b0] = Sl + off;
            off += e;
          } else {
            S[b] = hs[b - b0] = Sw + offw;
            offw += e;
          }
        }
        std::memcpy(h + o_ar, tAr.data() + bx0, 8 * (size_t)nbxl);
        std::memcpy(h + o_lar, lAr.data() + bx0, 8 * (size_t)nbxl);
        std::memcpy(h + o_ac, tAc.data() + by0, 8 * (size_t)nbyl);
        std::memcpy(h + o_lac, lAc.data() + by0, 8 * (size_t)nbyl);
        char* d = (char*)stage_launch(a, h, o_end);
        GformArgs ga{};
        ga.bt = d_bt;
        ga.tri_ptr = d_tptr;
        ga.tri = d_tri;
        ga.SX = d_tX;
        ga.ldSX = d_lX;
        ga.SY = d_tY;
        ga.ldSY = d_lY;
        ga.PS = fAA.B;
        ga.Ar = (const double* const*)(d + o_ar);
        ga.ldAr = (const int64_t*)(d + o_lar);
        ga.Ac = (const double* const*)(d + o_ac);
        ga.ldAc = (const int64_t*)(d + o_lac);
        ga.krow = (const int32_t*)d;
        ga.kcol = (const int32_t*)(d + o_kc);
        ga.Rr = (const double* const*)(d + o_rr);
        ga.Rc = (const double* const*)(d + o_rc);
        ga.S = (double* const*)(d + o_s);
        ga.b0 = b0;
        ga.c0 = c0;
        ga.bx0 = bx0;
        ga.by0 = by0;
        ga.k = k;
        ga.ktmax = ktmax;
        ga.krmax = krmax;
        LaunchTimer lt(a, KK_GEMM, flops, bytes);
        k_gform(ga, nb, prec, a->stream);
        continue;
      }
      const TriFamily fNA = family(d_tri, upload(a, tAr), upload(a, lAr), d_tY, d_lY, TK_NA, false,
                                   nullptr);  // A_{t,s} S_Y
      const TriFamily fAN = family(d_tri, d_tX, d_lX, upload(a, tAc), upload(a, lAc), TK_AN, true,
                                   nullptr);  // S_X A^c^*
      // couplings: admissible blocks in G, subdivided blocks in the
      // workspace until the top-down projections, dense leaves not stored
      // (folded into their blocks by the run that forms them)
      for (int b = b0; b < b1; ++b) {
        const int kt = row.Q.rank[B.t[b]], kr = col.Q.rank[B.s[b]];
        const size_t e = (size_t)std::max(kt, 1) * std::max(kr, 1);
        S[b] = B.type[b] == BT_ADM ? G->mem_nf.get<double>(e) : B.type[b] == BT_INADM ? nullptr : ws.get<double>(e);
      }
      // the level's blocks in runs whose scratch fits in run_scratch
      for (int cb0 = b0, cb1; cb0 < b1; cb0 = cb1) {
        size_t need = 0;
        for (cb1 = cb0; cb1 < b1; ++cb1) {
          const int kt = row.Q.rank[B.t[cb1]], kr = col.Q.rank[B.s[cb1]];
          size_t e = 8 * ((size_t)k * k + (size_t)kt * k + (size_t)k * kr) + 768;
          if (B.type[cb1] == BT_INADM)
            e += 8 * ((size_t)std::max(kt, 1) * std::max(kr, 1) + (size_t)T.size[B.t[cb1]] * kr) + 512;
          if (cb1 > cb0 && need + e > a->run_scratch) break;
          need += e;
        }
        unfused_run(cb0, cb1, fNA, fAN);
      }
    }
    step_end(a, 4);
  });
  // row pass (X, Y) here, column pass (Y^*, X^*) concurrently on the
  // auxiliary context; the two share only read-only inputs
  struct StopOnExit {
    LevelSignal& s;
    ~StopOnExit() { s.abort(); }
  } stop_on_exit{sig};
  G->mem_aux.bind(aux_ctx(ctx));
  {
    AuxRun colrun(ctx, [&](h2_ctx* a) { induced_pass(a, Yt, Xt, eps, G->mem_aux, col, 0, 3, &sig, 1); });
    induced_pass(ctx, X, Y, eps, G->mem, row, 0, 2, &sig, 0);
    colrun.join();
  }
  nfrun.join();
  G->n_triples = PT.n_terminated;

  // ---- G: the parents' S projected onto each block, top-down ----
  step_begin(ctx, 4);
  const BlockTreeH& B = *PT.bt;
  Arena& ws = ctx->ws;
  GemmBatch g;
  g.prec = prec;
  H2Core& C = G->c;
  C.ct = Xm->c.ct;
  C.bt = PT.bt;
  C.V = row.Q;
  C.W = col.Q;
  C.blk.assign(B.nblocks(), nullptr);
  // S_b += E_t S_parent F_r^* level by level (E, F: transfers of the new
  // bases); one fused launch per level, two grouped products where a rank
  // exceeds the fused kernel's 64
  Chain3Batch ch;
  // the two-step paths' middle products, in runs of at most run_scratch:
  // a run is flushed (chained products, first and second products) before
  // its scratch is reused
  ScopedArena tmp(ctx);
  std::vector<std::pair<int, double*>> wide;  // (block, middle product) of the two-step path
  size_t pend = 0;
  for (int l = 1; l <= T.depth; ++l) {
    const int b0 = B.lvl[l], b1 = B.lvl[l + 1];
    std::vector<int> parent(b1 - b0, -1);
    for (int pb = B.lvl[l - 1]; pb < b0; ++pb)
      if (B.type[pb] == BT_SPLIT)
        for (int q = 0; q < 4; ++q) parent[B.child0[pb] + q - b0] = pb;
    auto flush = [&] {  // S_b += (E_t S_parent) F_r^*
      ch.run(ctx);
      g.run(ctx);
      for (auto [b, Pp] : wide) {
        const int t = B.t[b], r = B.s[b], kt = row.Q.rank[t], kr = col.Q.rank[r];
        const int kpr = col.Q.rank[B.s[parent[b - b0]]];
        g.out(S[b], kt, kt, kr, true);
        g.term(Pp, kt, false, col.Q.tr[r], col.Q.tr_ld[r], true, kpr);
      }
      g.run(ctx);
      wide.clear();
      tmp.reset();
      pend = 0;
    };
    for (int b = b0; b < b1; ++b) {
      const int i = b - b0, t = B.t[b], r = B.s[b], kt = row.Q.rank[t], kr = col.Q.rank[r];
      if (parent[i] < 0 || kt == 0 || kr == 0 || !S[b]) continue;  // S[b] null: dense leaf, below
      const int pt = B.t[parent[i]], pr = B.s[parent[i]];
      const int kpt = row.Q.rank[pt], kpr = col.Q.rank[pr];
      if (kpt == 0 || kpr == 0) continue;
      if (Chain3Batch::fits(kt, kr, kpt, kpr)) {
        ch.add(S[b], kt, kt, kr, row.Q.tr[t], row.Q.tr_ld[t], false, kpt, S[parent[i]], kpt, kpr, col.Q.tr[r],
               col.Q.tr_ld[r], true, true);
        continue;
      }
      double* Pp = tmp.get<double>((size_t)kt * kpr);
      g.out(Pp, kt, kt, kpr);
      g.term(row.Q.tr[t], row.Q.tr_ld[t], false, S[parent[i]], kpt, false, kpt);
      wide.push_back({b, Pp});
      pend += 8 * (size_t)kt * kpr;
      if (pend > ctx->run_scratch) flush();
    }
    flush();
  }
  for (int b = 0; b < B.nblocks(); ++b)
    if (B.type[b] == BT_ADM) C.blk[b] = S[b];
  // dense inadmissible leaves: the nearfield products (already there) plus
  // Q_t S Q^W_r^*.  A leaf whose coupling was folded in when it was formed
  // (S[b] null) adds its parent's part (Q_t E_t) S_parent (Q^W_r F_r)^*.
  {
    const int l = T.depth;
    std::vector<int> parent(B.lvl[l + 1] - B.lvl[l], -1);
    if (l > 0)
      for (int pb = B.lvl[l - 1]; pb < B.lvl[l]; ++pb)
        if (B.type[pb] == BT_SPLIT)
          for (int q = 0; q < 4; ++q) parent[B.child0[pb] + q - B.lvl[l]] = pb;
    // Q_t E_t and Q^W_r F_r of the leaves that need them
    std::vector<double*> Wr(T.ncl, nullptr), Wc(T.ncl, nullptr);
    std::vector<std::pair<int, int>> folded;  // (block, parent) of the folded leaves with a parent part
    for (int b = B.lvl[l]; b < B.lvl[l + 1]; ++b) {
      if (B.type[b] != BT_INADM) continue;
      const int t = B.t[b], r = B.s[b];
      C.blk[b] = dense_block(t, r);
      const int pb = parent[b - B.lvl[l]];
      if (S[b] || pb < 0) continue;
      const int kt = row.Q.rank[t], kr = col.Q.rank[r], pt = B.t[pb], pr = B.s[pb];
      const int kpt = row.Q.rank[pt], kpr = col.Q.rank[pr];
      if (kt == 0 || kr == 0 || kpt == 0 || kpr == 0) continue;
      folded.push_back({b, pb});
      const int mt = (int)T.size[t], nr = (int)T.size[r];
      if (!Wr[t]) {
        Wr[t] = ws.get<double>((size_t)mt * kpt);
        g.out(Wr[t], mt, mt, kpt);
        g.term(row.Q.leaf[t], row.Q.leaf_ld[t], false, row.Q.tr[t], row.Q.tr_ld[t], false, kt);
      }
      if (!Wc[r]) {
        Wc[r] = ws.get<double>((size_t)nr * kpr);
        g.out(Wc[r], nr, nr, kpr);
        g.term(col.Q.leaf[r], col.Q.leaf_ld[r], false, col.Q.tr[r], col.Q.tr_ld[r], false, kr);
      }
    }
    g.run(ctx);
    auto flush = [&] {  // D += (Q_t S) Q^W_r^*, or D += ((Q_t E_t) S_parent) (Q^W_r F_r)^*
      ch.run(ctx);
      g.run(ctx);
      for (auto [b, P] : wide) {
        const int t = B.t[b], r = B.s[b], mt = (int)T.size[t], nr = (int)T.size[r];
        g.out(C.blk[b], mt, mt, nr, true);
        if (S[b])
          g.term(P, mt, false, col.Q.leaf[r], col.Q.leaf_ld[r], true, col.Q.rank[r]);
        else
          g.term(P, mt, false, Wc[r], nr, true, col.Q.rank[B.s[parent[b - B.lvl[l]]]]);
      }
      g.run(ctx);
      wide.clear();
      tmp.reset();
      pend = 0;
    };
    for (auto [b, pb] : folded) {
      const int t = B.t[b], mt = (int)T.size[t];
      const int kpt = row.Q.rank[B.t[pb]], kpr = col.Q.rank[B.s[pb]];
      double* P = tmp.get<double>((size_t)mt * kpr);
      g.out(P, mt, mt, kpr);
      g.term(Wr[t], mt, false, S[pb], kpt, false, kpt);
      wide.push_back({b, P});
      pend += 8 * (size_t)mt * kpr;
      if (pend > ctx->run_scratch) flush();
    }
    for (int b = B.lvl[l]; b < B.lvl[l + 1]; ++b) {
      if (B.type[b] != BT_INADM || !S[b]) continue;
      int t = B.t[b], r = B.s[b], kt = row.Q.rank[t], kr = col.Q.rank[r];
      double* Dn = C.blk[b];
      if (kt == 0 || kr == 0) continue;
      const int mt = (int)T.size[t], nr = (int)T.size[r];
      if (Chain3Batch::fits(mt, nr, kt, kr)) {
        ch.add(Dn, mt, mt, nr, row.Q.leaf[t], row.Q.leaf_ld[t], false, kt, S[b], kt, kr, col.Q.leaf[r],
               col.Q.leaf_ld[r], true, true);
        continue;
      }
      double* QS = tmp.get<double>((size_t)mt * kr);
      g.out(QS, mt, mt, kr);
      g.term(row.Q.leaf[t], row.Q.leaf_ld[t], false, S[b], kt, false, kt);
      wide.push_back({b, QS});
      pend += 8 * (size_t)mt * kr;
      if (pend > ctx->run_scratch) flush();
    }
    flush();
  }
  step_end(ctx, 4);
}

}  // namespace h2
