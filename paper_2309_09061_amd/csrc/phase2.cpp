// Phase 2: coarsening of G (an H^2-matrix on T^XY with isometric bases) into
// the prescribed block tree T_IK (Section 6, Figures "match_column" and
// "basis").  For the row basis (and on G* for the column basis):
//   top-down  product total weights Z_t from [Z_{t+} E_t^*; S_{t,r}^*] over
//             the admissible leaves of T^XY inside admissible leaves of T_IK
//             (eq. (Zt_condensation));
//   bottom-up leaf clusters: C_t = [V_t Z_t^*, G|_{t x r_i}] (eq. (ct_leaf));
//             non-leaf clusters: Chat_t = [Vhat_t Z_t^*, Ahat_{t,r_i}]
//             (eq. (ct_nonleaf)), Ahat assembled from the children's
//             representations on the column tree of (t, r_i) (Definition
//             "Column tree", Lemma "Column representation", Figure
//             "match_column"); SVD and rank choice at eps; R_t = Q_t^* V_t
//             and A_{t,r} = Q_t^* G|_{t x r}.
// Every block is scaled by omega_b = 1/||G|_b||_F of the admissible leaf b
// of T_IK containing it.  Z's couplings Q^Z_t^* G|_b Q^ZW_r are accumulated
// bottom-up over the blocks of T^XY inside b; Z's nearfield copies G.
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <unordered_map>

#include "internal.h"

namespace h2 {

struct ColLeaf {
  int32_t node;
  int32_t adm;
  int32_t width;
  int32_t off;
};

struct P2Side {
  Basis Q;                   // new basis (leaf matrices and transfers)
  std::vector<double*> R;    // R_t = Q_t^* V_t: kz_t x k_t, ld max(kz_t, 1)
  std::vector<double*> A;    // per stored G block: A_{t,r} (kz_t x width), ld max(kz_t, 1)
  std::vector<double*> RS;   // per stored admissible G leaf: R_t S_{t,r}, kz_t x kW_r
  std::vector<double*> RZ;   // Z != 0: Q_t^* V^Z_t (the old Z's basis in the new one), kz_t x kold_t
};

// Column trees of all blocks in one array (per pass): the leaves of block b
// are leaves[beg[b] .. beg[b] + len[b]), ordered by position.
struct ColTrees {
  std::vector<ColLeaf> leaves;
  std::vector<int64_t> beg;
  std::vector<int32_t> len;
};

// appends the union of the leaf lists of blocks c1 and c2 (which cover the
// same index range) to the array
static void leaf_union_into(const TreeH& T, ColTrees& C, int c1, int c2) {
  const int64_t a = C.beg[c1], b = C.beg[c2];
  const int na = C.len[c1], nb = C.len[c2];
  int i = 0, j = 0;
  while (i < na && j < nb) {
    const ColLeaf x = C.leaves[a + i], y = C.leaves[b + j];
    if (x.node == y.node) {
      C.leaves.push_back({x.node, x.adm && y.adm, 0, 0});
      ++i;
      ++j;
    } else if (T.size[x.node] < T.size[y.node]) {  // x lies inside y
      C.leaves.push_back(x);
      if (T.off[x.node] + T.size[x.node] == T.off[y.node] + T.size[y.node]) ++j;
      ++i;
    } else {
      C.leaves.push_back(y);
      if (T.off[x.node] + T.size[x.node] == T.off[y.node] + T.size[y.node]) ++i;
      ++j;
    }
  }
  H2_REQUIRE(i == na && j == nb, H2_ERR_SHAPE, "column trees do not cover one range");
}

// Kb: for Z <- Z + G with Z != 0, the old Z's basis on this side (row
// basis for the row pass, column basis for the column pass), whose range is
// kept exactly (as phase 1 keeps range(V_X)); null for Z = 0.
static void coarse_pass(h2_ctx* ctx, const View& G, const std::vector<int>& tag,
                        const BlockTreeH& TIK, const double* omega, double eps, Arena& keep,
                        P2Side& out, int step, const Basis* Kb) {
  const TreeH& T = *G.m->ct;
  const BlockTreeH& B = G.bt();
  const int ncl = T.ncl, D = T.depth, nb = B.nblocks();
  const Basis& Vb = G.rowb();
  const Basis& Wb = G.colb();
  Arena& ws = ctx->ws;
  GemmBatch g;
  g.prec = ctx->prec;
  step_begin(ctx, step);
  auto in_adm = [&](int b) { return tag[b] >= 0 && TIK.type[tag[b]] == BT_ADM; };
  const double* om = omega;  // omega + tag[b] is the scale of block b

  // ---- product total weights Z_t, top-down ----
  std::vector<double*> Zt(ncl, nullptr);
  std::vector<int> zr(ncl, 0);
  // per-level temporaries (the stacked weights here, C_t and its factors in
  // the sweep below): one level at a time
  ScopedArena lvl(ctx);
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
    for (int t = T.first(l); t < T.first(l + 1); ++t) {
      int kt = Vb.rank[t];
      int zp = l > 0 ? zr[TreeH::parent(t)] : 0;
      int N = zp;
      const int32_t* bl;
      int cnt;
      G.row_blocks(t, bl, cnt);
      for (int q = 0; q < cnt; ++q)
        if (B.type[bl[q]] == BT_ADM && in_adm(bl[q])) N += Wb.rank[G.vcol(bl[q])];
      Zt[t] = ws.get<double>((size_t)std::max(kt, 1) * std::max(kt, 1));
      zr[t] = std::min(N, kt);
      if (N == 0 || kt == 0) {
        zr[t] = 0;
        continue;
      }
      const size_t e = 8 * (size_t)N * kt;
      if (pend > 0 && pend + e > ctx->run_scratch) flush();
      double* Gh = lvl.get<double>((size_t)N * kt);
      pend += e;
      int row = 0;
      if (zp > 0) {
        int kp = Vb.rank[TreeH::parent(t)];
        g.out(Gh, N, zp, kt);
        g.term(Zt[TreeH::parent(t)], std::max(kp, 1), false, Vb.tr[t], Vb.tr_ld[t], true, kp);
        row += zp;
      }
      for (int q = 0; q < cnt; ++q) {
        int b = bl[q];
        if (B.type[b] != BT_ADM || !in_adm(b)) continue;
        int kw = Wb.rank[G.vcol(b)];
        if (kw == 0) continue;
        g.out(Gh + row, N, kw, kt);
        g.copy(G.ptr(b), G.ld(b), !G.T, kt, 1.0, om + tag[b], 1);  // omega S_{t,r}^*
        row += kw;
      }
      ts.add(Gh, N, N, kt, false, Zt[t], std::max(kt, 1));
    }
    flush();
  }

  // Column trees (leaf lists over the view column) of blocks inside
  // admissible leaves of T_IK, the transfer chains of the column basis used
  // by match_column and W_a restricted to leaves: host work and a few small
  // products, done while the device factorizes the leaf level
  ColTrees ct;
  ct.beg.assign(nb, 0);
  ct.len.assign(nb, 0);
  auto tree_width = [&](int b) {
    if (ct.len[b] == 0) return 0;
    const ColLeaf& e = ct.leaves[ct.beg[b] + ct.len[b] - 1];
    return e.off + e.width;
  };
  std::unordered_map<int64_t, std::pair<const double*, int64_t>> chain;
  auto key = [&](int c, int a) { return (int64_t)c * ncl + a; };
  std::function<void(int, int)> need;
  std::vector<std::vector<std::pair<int, int>>> by_dist(D + 2);
  struct Piece {
    int blk, tc, src, srcoff, srcld, snode, sadm, tnode, tadm, twidth, toff, roff;
    int rowpos;  // position of blk in the block list of its row
  };
  std::vector<std::vector<Piece>> pieces(D + 1);
  std::unordered_map<int64_t, std::pair<const double*, int64_t>> wrest;
  auto build_columns = [&]() {
    for (int l = D; l >= 0; --l)
      for (int b = B.lvl[l]; b < B.lvl[l + 1]; ++b) {
        if (!in_adm(b)) continue;
        int r = G.vcol(b), t = G.vrow(b);
        ct.beg[b] = (int64_t)ct.leaves.size();
        if (B.type[b] != BT_SPLIT) {
          ct.leaves.push_back({r, B.type[b] == BT_ADM ? 1 : 0, 0, 0});
        } else {
          for (int qc = 1; qc <= 2; ++qc) {
            int rc = 2 * r + qc;
            int c1 = G.find(2 * t + 1, rc), c2 = G.find(2 * t + 2, rc);
            H2_REQUIRE(c1 >= 0 && c2 >= 0, H2_ERR_SHAPE, "product tree: missing child");
            leaf_union_into(T, ct, c1, c2);
          }
        }
        ct.len[b] = (int32_t)((int64_t)ct.leaves.size() - ct.beg[b]);
        int off = 0;
        for (int64_t e = ct.beg[b]; e < ct.beg[b] + ct.len[b]; ++e) {
          ColLeaf& L = ct.leaves[e];
          L.width = L.adm ? Wb.rank[L.node] : (int)T.size[L.node];
          L.off = off;
          off += L.width;
        }
      }

    // ---- transfer chains of the column basis used by match_column ----
    // CH(c, a) = F_c F_{parent(c)} ... : W_a restricted to c equals W_c CH(c, a)
    need = [&](int c, int a) {
      if (chain.count(key(c, a))) return;
      int p = TreeH::parent(c);
      if (p == a) {
        chain[key(c, a)] = {Wb.tr[c], Wb.tr_ld[c]};
        return;
      }
      need(p, a);
      chain[key(c, a)] = {nullptr, 0};
      by_dist[TreeH::level(c) - TreeH::level(a)].push_back({c, a});
    };
    auto contains = [&](int a, int c) {  // cluster a contains cluster c
      return T.off[a] <= T.off[c] && T.off[c] + T.size[c] <= T.off[a] + T.size[a] && TreeH::level(a) <= TreeH::level(c);
    };
    for (int l = 0; l < D; ++l)
      for (int b = B.lvl[l]; b < B.lvl[l + 1]; ++b) {
        if (B.type[b] != BT_SPLIT || !in_adm(b)) continue;
        int t = G.vrow(b), r = G.vcol(b);
        int rowpos = 0;
        {
          const int32_t* bl;
          int cnt;
          G.row_blocks(t, bl, cnt);
          while (rowpos < cnt && bl[rowpos] != b) ++rowpos;
        }
        for (int64_t e = ct.beg[b]; e < ct.beg[b] + ct.len[b]; ++e) {
          const ColLeaf& L = ct.leaves[e];
          int rc = contains(2 * r + 1, L.node) ? 2 * r + 1 : 2 * r + 2;
          for (int qt = 1; qt <= 2; ++qt) {
            int tc = 2 * t + qt;
            int c = G.find(tc, rc);
            // the last leaf of c's column tree containing L; the list is
            // ordered by position, so no leaf after the last one starting at
            // or before L can contain it (the backward scan only moves past
            // empty clusters)
            const ColLeaf* c_beg = ct.leaves.data() + ct.beg[c];
            const ColLeaf* c_end = c_beg + ct.len[c];
            const ColLeaf* it = std::upper_bound(c_beg, c_end, T.off[L.node],
                                                 [&](int64_t o, const ColLeaf& M) { return o < T.off[M.node]; });
            const ColLeaf* S = nullptr;
            while (it != c_beg && !S) {
              --it;
              if (contains(it->node, L.node)) S = it;
            }
            H2_REQUIRE(S, H2_ERR_SHAPE, "match_column: no source leaf");
            H2_REQUIRE(S->adm || S->node == L.node, H2_ERR_UNSUPPORTED,
                       "match_column: inadmissible column leaf refined");
            pieces[l].push_back({b, tc, c, S->off, 0, S->node, S->adm, L.node, L.adm, L.width, L.off, qt, rowpos});
            if (S->adm && S->node != L.node) need(L.node, S->node);
          }
        }
      }
    for (int d = 2; d <= D + 1; ++d) {
      if (d >= (int)by_dist.size() || by_dist[d].empty()) continue;
      for (auto [c, a] : by_dist[d]) {
        int p = TreeH::parent(c);
        auto pr = chain[key(p, a)];
        double* M = ws.get<double>((size_t)std::max(Wb.rank[c], 1) * std::max(Wb.rank[a], 1));
        g.out(M, std::max(Wb.rank[c], 1), Wb.rank[c], Wb.rank[a]);
        g.term(Wb.tr[c], Wb.tr_ld[c], false, pr.first, pr.second, false, Wb.rank[p]);
        chain[key(c, a)] = {M, std::max(Wb.rank[c], 1)};
      }
      g.run(ctx);
    }
    // W_{a} restricted to the leaf c: Q^W_c CH(c, a)
    for (int l = 0; l < D; ++l)
      for (const Piece& P : pieces[l]) {
        if (!P.sadm || P.tadm) continue;
        int64_t kk = key(P.tnode, P.snode);
        if (wrest.count(kk)) continue;
        if (P.tnode == P.snode) {
          wrest[kk] = {Wb.leaf[P.tnode], Wb.leaf_ld[P.tnode]};
          continue;
        }
        auto ch = chain[key(P.tnode, P.snode)];
        double* M = ws.get<double>((size_t)T.size[P.tnode] * std::max(Wb.rank[P.snode], 1));
        g.out(M, T.size[P.tnode], (int)T.size[P.tnode], Wb.rank[P.snode]);
        g.term(Wb.leaf[P.tnode], Wb.leaf_ld[P.tnode], false, ch.first, ch.second, false, Wb.rank[P.tnode]);
        wrest[kk] = {M, T.size[P.tnode]};
      }
    g.run(ctx);
  };

  // ---- Figure "basis", bottom-up ----
  out.Q.resize(ncl);
  out.R.assign(ncl, nullptr);
  out.A.assign(nb, nullptr);
  out.RS.assign(nb, nullptr);
  out.RZ.assign(ncl, nullptr);
  for (int l = D; l >= 0; --l) {
    lvl.reset();
    const int c0 = T.first(l), c1 = T.first(l + 1), nc = c1 - c0;
    const bool leaf = l == D;
    std::vector<int> m(nc), ncols(nc);
    std::vector<double*> Vh(nc, nullptr), C(nc), Rt(nc, nullptr), U(nc, nullptr), sg(nc, nullptr);
    std::vector<std::vector<int>> cols_of(nc);
    // Vhat_t = [R_{t'} E_{t'}]
    for (int i = 0; i < nc; ++i) {
      int t = c0 + i, kt = Vb.rank[t];
      if (leaf) {
        m[i] = (int)T.size[t];
        continue;
      }
      int o = 0;
      m[i] = out.Q.rank[2 * t + 1] + out.Q.rank[2 * t + 2];
      Vh[i] = lvl.get<double>((size_t)std::max(m[i], 1) * std::max(kt, 1));
      for (int q = 1; q <= 2; ++q) {
        int ch = 2 * t + q, kc = out.Q.rank[ch];
        if (kc > 0) {
          g.out(Vh[i] + o, m[i], kc, kt);
          g.term(out.R[ch], kc, false, Vb.tr[ch], Vb.tr_ld[ch], false, Vb.rank[ch]);
        }
        o += kc;
      }
    }
    g.run(ctx);
    // C_t / Chat_t.  Without an old Z, the leaves' C_t are needed only for
    // their R factors: they are built and reduced in runs below, so that the
    // level holds one run of them at a time.
    const bool stream_leaf = leaf && !Kb;
    auto fill_C = [&](int i, Arena& ar) {
      const int t = c0 + i, kt = Vb.rank[t];
      C[i] = ar.get<double>((size_t)std::max(m[i], 1) * std::max(ncols[i], 1));
      if (m[i] == 0) return;
      if (zr[t] > 0) {
        g.out(C[i], m[i], m[i], zr[t]);
        if (leaf)
          g.term(Vb.leaf[t], Vb.leaf_ld[t], false, Zt[t], std::max(kt, 1), true, kt);
        else
          g.term(Vh[i], m[i], false, Zt[t], std::max(kt, 1), true, kt);
      }
      if (leaf) {
        const int32_t* bl;
        int cnt;
        G.row_blocks(t, bl, cnt);
        for (int q = 0; q < cnt; ++q) {
          int b = bl[q];
          if (cols_of[i][q] < 0) continue;
          int r = G.vcol(b);
          g.out(C[i] + (size_t)cols_of[i][q] * m[i], m[i], m[i], (int)T.size[r]);
          g.copy(G.ptr(b), G.ld(b), G.T, (int)T.size[r], 1.0, om + tag[b], 1);
        }
      }
    };
    for (int i = 0; i < nc; ++i) {
      int t = c0 + i, kt = Vb.rank[t];
      const int32_t* bl;
      int cnt;
      G.row_blocks(t, bl, cnt);
      int nco = zr[t];
      for (int q = 0; q < cnt; ++q) {
        int b = bl[q];
        if (!in_adm(b)) {
          cols_of[i].push_back(-1);
        } else if (leaf && B.type[b] == BT_INADM) {
          cols_of[i].push_back(nco);
          nco += (int)T.size[G.vcol(b)];
        } else if (!leaf && B.type[b] == BT_SPLIT) {
          cols_of[i].push_back(nco);
          nco += tree_width(b);
        } else {
          cols_of[i].push_back(-1);
        }
      }
      ncols[i] = nco;
      if (!stream_leaf) fill_C(i, lvl);
    }
    if (!leaf) {
      // Ahat_{t,r}: the children's representations matched to the column tree of (t,r)
      for (const Piece& P : pieces[l]) {
        int t = G.vrow(P.blk), i = t - c0;
        int kc = out.Q.rank[P.tc];
        if (kc == 0) continue;
        int ro = P.roff == 1 ? 0 : out.Q.rank[2 * t + 1];
        double* dst = C[i] + ro + (size_t)(cols_of[i][P.rowpos] + P.toff) * m[i];
        const double* src;
        int64_t sld = std::max(kc, 1);
        if (B.type[P.src] == BT_ADM)
          src = out.RS[P.src];
        else
          src = out.A[P.src] + (size_t)P.srcoff * sld;
        g.out(dst, m[i], kc, P.twidth);
        const double* sc = om + tag[P.blk];
        if (!P.sadm) {
          g.copy(src, sld, false, P.twidth, 1.0, sc, 1);
        } else if (P.tadm) {
          if (P.snode == P.tnode)
            g.copy(src, sld, false, P.twidth, 1.0, sc, 1);
          else {
            auto ch = chain[key(P.tnode, P.snode)];
            g.term(src, sld, false, ch.first, ch.second, true, Wb.rank[P.snode], 1.0, sc, 1);
          }
        } else {
          auto wr = wrest[key(P.tnode, P.snode)];
          g.term(src, sld, false, wr.first, wr.second, true, Wb.rank[P.snode], 1.0, sc, 1);
        }
      }
    }
    g.run(ctx);
    std::vector<int32_t> kz(nc, 0);
    std::vector<double*> Qk(nc, nullptr);
    if (Kb) {
      // Z != 0: keep range(V^Z_t) (leaf) or range(Vhat^Z_t = [RZ_{t'} E^Z_{t'}]),
      // truncate the rest of C_t (a copy: the inner levels read C_t below)
      std::vector<KeptItem> kit(nc);
      for (int i = 0; i < nc; ++i) {
        int t = c0 + i, kold = Kb->rank[t];
        const double* K = nullptr;
        int64_t ldk = std::max(m[i], 1);
        if (leaf) {
          K = Kb->leaf[t];
          ldk = Kb->leaf_ld[t];
        } else if (m[i] > 0 && kold > 0) {
          double* Kh = lvl.get<double>((size_t)m[i] * kold);
          int o = 0;
          for (int q = 1; q <= 2; ++q) {
            int ch = 2 * t + q, kc = out.Q.rank[ch];
            if (kc > 0) {
              g.out(Kh + o, m[i], kc, kold);
              if (Kb->rank[ch] > 0)
                g.term(out.RZ[ch], kc, false, Kb->tr[ch], Kb->tr_ld[ch], false, Kb->rank[ch]);
            }
            o += kc;
          }
          K = Kh;
        }
        double* Cw = lvl.get<double>((size_t)std::max(m[i], 1) * std::max(ncols[i], 1));
        if (m[i] > 0 && ncols[i] > 0) {
          g.out(Cw, m[i], m[i], ncols[i]);
          g.copy(C[i], m[i], false, ncols[i]);
        }
        kit[i] = {m[i], K, ldk, K ? kold : 0, Cw, std::max(m[i], 1), ncols[i]};
      }
      g.run(ctx);
      KeptOut ko;
      if (leaf) build_columns();  // host work while the device factorizes
      kept_compress(ctx, kit, level_eps(ctx, eps, D, l), keep, ko);
      for (int i = 0; i < nc; ++i) {
        kz[i] = ko.k1[i] + ko.k2[i];
        Qk[i] = ko.Q[i];
        out.RZ[c0 + i] = ko.RKP[i];
      }
    } else {
      // SVD of C_t: R factor of C_t^*, one-sided Jacobi
      TsqrBatch ts;
      JacobiBatch jb;
      int32_t* rk = lvl.get<int32_t>(nc);
      dev_zero(rk, sizeof(int32_t) * nc, ctx->stream);
      for (int i = 0; i < nc; ++i) {
        if (m[i] == 0) continue;
        int p = std::min(ncols[i], m[i]);
        Rt[i] = lvl.get<double>((size_t)m[i] * m[i]);  // rows < p are written
        U[i] = lvl.get<double>((size_t)m[i] * m[i]);
        sg[i] = lvl.get<double>(m[i]);
        if (!stream_leaf) ts.add(C[i], m[i], ncols[i], m[i], true, Rt[i], m[i]);
        jb.add(Rt[i], m[i], p, m[i], U[i], m[i], sg[i], rk + i, level_eps(ctx, eps, D, l), 0.0, nullptr, 1,
               ctx->rank_rule);
      }
      if (stream_leaf) {
        // runs of at most run_scratch bytes of C_t: built, then reduced to
        // their R factors, before the run's memory is reused
        ScopedArena run(ctx);
        size_t pend = 0;
        auto flush = [&] {
          g.run(ctx);
          ts.run(ctx);
          run.reset();
          pend = 0;
        };
        for (int i = 0; i < nc; ++i) {
          if (m[i] == 0) continue;
          const size_t e = 8 * (size_t)m[i] * std::max(ncols[i], 1);
          if (pend > 0 && pend + e > ctx->run_scratch) flush();
          fill_C(i, run);
          pend += e;
          ts.add(C[i], m[i], ncols[i], m[i], true, Rt[i], m[i]);
        }
        flush();
      } else {
        ts.run(ctx);
      }
      jb.run(ctx);
      const int32_t* kzh = read_back(ctx, rk, nc);
      if (leaf) build_columns();
      ctx_sync(ctx);
      for (int i = 0; i < nc; ++i) kz[i] = kzh[i];
    }
    // new basis, R_t, A_{t,r}
    for (int i = 0; i < nc; ++i) {
      int t = c0 + i, kt = Vb.rank[t], k = kz[i];
      out.Q.rank[t] = k;
      double* Qn = Qk[i];
      if (!Qn) {
        Qn = keep.get<double>((size_t)std::max(m[i], 1) * std::max(k, 1));
        if (k > 0) {
          g.out(Qn, m[i], m[i], k);
          g.copy(U[i], m[i], false, k);
        }
      }
      if (leaf) {
        out.Q.leaf[t] = Qn;
        out.Q.leaf_ld[t] = std::max(m[i], 1);
      } else {
        out.Q.tr[2 * t + 1] = Qn;
        out.Q.tr[2 * t + 2] = Qn + out.Q.rank[2 * t + 1];
        out.Q.tr_ld[2 * t + 1] = out.Q.tr_ld[2 * t + 2] = std::max(m[i], 1);
      }
      out.R[t] = ws.get<double>((size_t)std::max(k, 1) * std::max(kt, 1));
    }
    g.run(ctx);
    for (int i = 0; i < nc; ++i) {
      int t = c0 + i, kt = Vb.rank[t], k = out.Q.rank[t];
      double* Qn = leaf ? out.Q.leaf[t] : out.Q.tr[2 * t + 1];
      if (k > 0 && kt > 0) {
        g.out(out.R[t], k, k, kt);
        if (leaf)
          g.term(Qn, m[i], true, Vb.leaf[t], Vb.leaf_ld[t], false, m[i]);
        else
          g.term(Qn, m[i], true, Vh[i], m[i], false, m[i]);
      }
      const int32_t* bl;
      int cnt;
      G.row_blocks(t, bl, cnt);
      for (int q = 0; q < cnt; ++q) {
        int b = bl[q];
        if (!in_adm(b)) continue;
        if (cols_of[i][q] >= 0) {
          int w = leaf ? (int)T.size[G.vcol(b)] : tree_width(b);
          out.A[b] = ws.get<double>((size_t)std::max(k, 1) * std::max(w, 1));
          if (k == 0) continue;
          g.out(out.A[b], k, k, w);
          if (leaf)
            g.term(Qn, m[i], true, G.ptr(b), G.ld(b), G.T, m[i]);  // Q_t^* G|_{t x r}
          else
            g.term(Qn, m[i], true, C[i] + (size_t)cols_of[i][q] * m[i], m[i], false, m[i], 1.0,
                   om + tag[b], 2);
        }
      }
    }
    g.run(ctx);
    // R_t S_{t,r} for admissible leaves of this level (used above and for Z)
    for (int i = 0; i < nc; ++i) {
      int t = c0 + i, k = out.Q.rank[t], kt = Vb.rank[t];
      const int32_t* bl;
      int cnt;
      G.row_blocks(t, bl, cnt);
      for (int q = 0; q < cnt; ++q) {
        int b = bl[q];
        if (B.type[b] != BT_ADM || !in_adm(b)) continue;
        int kw = Wb.rank[G.vcol(b)];
        out.RS[b] = ws.get<double>((size_t)std::max(k, 1) * std::max(kw, 1));
        if (k == 0 || kw == 0) continue;
        g.out(out.RS[b], k, k, kw);
        g.term(out.R[t], k, false, G.ptr(b), G.ld(b), G.T, kt);
      }
    }
    g.run(ctx);
  }
  step_end(ctx, step);
}

void phase2(h2_ctx* ctx, h2_product* Gp, h2_matrix* Z, double eps, int prec) {
  const TreeH& T = *Gp->c.ct;
  H2_REQUIRE(T.same_as(*Z->c.ct), H2_ERR_SHAPE, "Z must be built on the cluster tree of X and Y");
  ctx->prec = prec;
  const BlockTreeH& B = *Gp->c.bt;
  const BlockTreeH& TIK = *Z->c.bt;
  const int nb = B.nblocks();
  // T_IK leaf containing each block of T^XY (-1: the block is a non-leaf of
  // T_IK), by one pass from the root: same[b] is the block of T_IK equal to
  // b (-1 below a leaf of T_IK); the four children of a subdivided block
  // are matched among the four children of its T_IK block
  std::vector<int> tag(nb, -1), same(nb, -1);
  same[0] = TIK.find(B.t[0], B.s[0]);
  H2_REQUIRE(same[0] >= 0, H2_ERR_NOT_REFINED, "T^XY does not refine T_IK");
  for (int b = 0; b < nb; ++b) {  // parents before children
    const int f = same[b];
    if (f >= 0) tag[b] = TIK.type[f] == BT_SPLIT ? -1 : f;
    if (B.type[b] != BT_SPLIT) {
      H2_REQUIRE(tag[b] >= 0, H2_ERR_NOT_REFINED, "T^XY does not refine T_IK");
      continue;
    }
    for (int q = 0; q < 4; ++q) {
      const int c = B.child0[b] + q;
      if (f >= 0 && TIK.type[f] == BT_SPLIT) {
        for (int qq = 0; qq < 4; ++qq) {
          const int cc = TIK.child0[f] + qq;
          if (TIK.t[cc] == B.t[c] && TIK.s[cc] == B.s[c]) same[c] = cc;
        }
        H2_REQUIRE(same[c] >= 0, H2_ERR_NOT_REFINED, "T^XY does not refine T_IK");
      } else {
        tag[c] = tag[b];
      }
    }
  }
  // omega_b = 1/||G|_b||_F over the leaves of T^XY inside admissible b:
  // the leaves grouped by their T_IK block (counting sort, in block order)
  auto in_sum = [&](int b) {
    return B.type[b] != BT_SPLIT && tag[b] >= 0 && TIK.type[tag[b]] == BT_ADM && Gp->c.blk[b];
  };
  std::vector<int32_t> sp(TIK.nblocks() + 1, 0);
  for (int b = 0; b < nb; ++b)
    if (in_sum(b)) ++sp[tag[b] + 1];
  for (int i = 0; i < TIK.nblocks(); ++i) sp[i + 1] += sp[i];
  std::vector<SumsqItem> items(std::max(sp.back(), 1), SumsqItem{nullptr, 1, 0, 0});
  {
    std::vector<int32_t> pos(sp.begin(), sp.end() - 1);
    for (int b = 0; b < nb; ++b) {
      if (!in_sum(b)) continue;
      int rows = B.type[b] == BT_ADM ? Gp->c.V.rank[B.t[b]] : (int)T.size[B.t[b]];
      int cols = B.type[b] == BT_ADM ? Gp->c.W.rank[B.s[b]] : (int)T.size[B.s[b]];
      items[pos[tag[b]]++] = {Gp->c.blk[b], Gp->c.ld_of(b), rows, cols};
    }
  }
  double* omega = ctx->ws.get<double>(std::max(TIK.nblocks(), 1));
  k_sumsq(upload(ctx, items), upload(ctx, sp), TIK.nblocks(), omega, 1, ctx->stream);

  View Gr{&Gp->c, false}, Gc{&Gp->c, true};
  // Z <- Z + G: a non-zero Z keeps the ranges of its bases (the passes keep
  // them exactly), its couplings are written in the new bases and its
  // nearfield is added; the new Z is built in fresh arenas and replaces the
  // old one at the end
  const bool add_old = !Z->zero;
  H2Core old;
  if (add_old) old = Z->c;
  Arena nmem, naux;
  nmem.bind(ctx);
  naux.bind(aux_ctx(ctx));
  // row pass on G here, column pass on G^* concurrently on the auxiliary
  // context; both read G, tag, omega and the old Z only
  P2Side row, col;
  {
    AuxRun colrun(ctx, [&](h2_ctx* a) {
      coarse_pass(a, Gc, tag, TIK, omega, eps, naux, col, 6, add_old ? &old.W : nullptr);
    });
    coarse_pass(ctx, Gr, tag, TIK, omega, eps, nmem, row, 5, add_old ? &old.V : nullptr);
    colrun.join();
  }

  // ---- Z: couplings Q^Z_t^* G|_b Q^ZW_r bottom-up, nearfield copied ----
  step_begin(ctx, 7);
  Arena& ws = ctx->ws;
  GemmBatch g;
  g.prec = prec;
  H2Core Zc = Z->c;  // assigned to Z at the end (Z is untouched on an error)
  Zc.V = row.Q;
  Zc.W = col.Q;
  Zc.blk.assign(TIK.nblocks(), nullptr);
  const Basis &QZ = row.Q, &QZW = col.Q;
  std::vector<double*> L(nb, nullptr);
  for (int l = T.depth; l >= 0; --l) {
    std::vector<double*> T1(nb, nullptr);
    for (int b = B.lvl[l]; b < B.lvl[l + 1]; ++b) {
      if (tag[b] < 0 || TIK.type[tag[b]] != BT_ADM) continue;
      int t = B.t[b], r = B.s[b], kz = QZ.rank[t], kw = QZW.rank[r];
      bool top = same[b] >= 0 && same[b] == tag[b];  // b is the T_IK leaf itself
      L[b] = top ? nmem.get<double>((size_t)std::max(kz, 1) * std::max(kw, 1))
                 : ws.get<double>((size_t)std::max(kz, 1) * std::max(kw, 1));
      if (B.type[b] == BT_SPLIT)
        for (int q = 0; q < 4; ++q) {
          int c = B.child0[b] + q, tc = B.t[c], rc = B.s[c];
          T1[c] = ws.get<double>((size_t)std::max(QZ.rank[tc], 1) * std::max(kw, 1));
          if (QZ.rank[tc] == 0 || kw == 0) continue;
          g.out(T1[c], QZ.rank[tc], QZ.rank[tc], kw);
          g.term(L[c], std::max(QZ.rank[tc], 1), false, QZW.tr[rc], QZW.tr_ld[rc], false, QZW.rank[rc]);
        }
    }
    g.run(ctx);
    for (int b = B.lvl[l]; b < B.lvl[l + 1]; ++b) {
      if (tag[b] < 0 || TIK.type[tag[b]] != BT_ADM) continue;
      int t = B.t[b], r = B.s[b], kz = QZ.rank[t], kw = QZW.rank[r];
      if (kz == 0 || kw == 0) continue;
      g.out(L[b], kz, kz, kw);
      if (B.type[b] == BT_ADM) {
        // R_t S_tr R^W_r^*
        g.term(row.RS[b], kz, false, col.R[r], kw, true, Gp->c.W.rank[r]);
      } else if (B.type[b] == BT_INADM) {
        // (Q^Z_t^* N_tr) Q^ZW_r
        g.term(row.A[b], kz, false, QZW.leaf[r], QZW.leaf_ld[r], false, (int)T.size[r]);
      } else {
        for (int q = 0; q < 4; ++q) {
          int c = B.child0[b] + q, tc = B.t[c];
          g.term(QZ.tr[tc], QZ.tr_ld[tc], true, T1[c], std::max(QZ.rank[tc], 1), false, QZ.rank[tc]);
        }
      }
    }
    g.run(ctx);
  }
  std::vector<int> of_tik(TIK.nblocks(), -1);  // the block of T^XY equal to a T_IK block
  for (int b = 0; b < nb; ++b)
    if (same[b] >= 0) of_tik[same[b]] = b;
  if (add_old) {
    // the old couplings in the new bases: L_b += RZ_t S^old_b RZW_r^*
    std::vector<double*> T1(TIK.nblocks(), nullptr);
    for (int zb = 0; zb < TIK.nblocks(); ++zb) {
      if (TIK.type[zb] != BT_ADM || !old.blk[zb]) continue;
      int t = TIK.t[zb], r = TIK.s[zb], kz = QZ.rank[t], ko = old.V.rank[t], kor = old.W.rank[r];
      if (kz == 0 || ko == 0 || kor == 0) continue;
      T1[zb] = ws.get<double>((size_t)kz * kor);
      g.out(T1[zb], kz, kz, kor);
      g.term(row.RZ[t], kz, false, old.blk[zb], old.ld_of(zb), false, ko);
    }
    g.run(ctx);
    for (int zb = 0; zb < TIK.nblocks(); ++zb) {
      if (!T1[zb]) continue;
      int t = TIK.t[zb], r = TIK.s[zb], kz = QZ.rank[t], kw = QZW.rank[r], kor = old.W.rank[r];
      const int b = of_tik[zb];
      H2_REQUIRE(b >= 0 && L[b], H2_ERR_NOT_REFINED, "admissible leaf of T_IK missing from T^XY");
      if (kw == 0) continue;
      g.out(L[b], kz, kz, kw, true);
      g.term(T1[zb], kz, false, col.RZ[r], std::max(kw, 1), true, kor);
    }
    g.run(ctx);
  }
  for (int zb = 0; zb < TIK.nblocks(); ++zb) {
    if (TIK.type[zb] == BT_SPLIT) continue;
    int t = TIK.t[zb], r = TIK.s[zb];
    int b = of_tik[zb];
    H2_REQUIRE(b >= 0, H2_ERR_NOT_REFINED, "leaf of T_IK missing from T^XY");
    if (TIK.type[zb] == BT_ADM) {
      Zc.blk[zb] = L[b];
    } else {
      double* Nz = nmem.get<double>((size_t)T.size[t] * T.size[r]);
      Zc.blk[zb] = Nz;
      g.out(Nz, T.size[t], (int)T.size[t], (int)T.size[r]);
      if (B.type[b] == BT_INADM) {
        g.copy(Gp->c.blk[b], Gp->c.ld_of(b), false, (int)T.size[r]);
      } else {
        H2_REQUIRE(B.type[b] == BT_ADM, H2_ERR_NOT_REFINED, "inadmissible leaf of T_IK subdivided in T^XY");
        int kt = Gp->c.V.rank[t], kr = Gp->c.W.rank[r];
        double* QS = ws.get<double>((size_t)T.size[t] * std::max(kr, 1));
        GemmBatch g0;
        g0.prec = prec;
        g0.out(QS, T.size[t], (int)T.size[t], kr);
        g0.term(Gp->c.V.leaf[t], Gp->c.V.leaf_ld[t], false, Gp->c.blk[b], Gp->c.ld_of(b), false, kt);
        g0.run(ctx);
        g.term(QS, T.size[t], false, Gp->c.W.leaf[r], Gp->c.W.leaf_ld[r], true, kr);
      }
      if (add_old && old.blk[zb]) g.copy(old.blk[zb], old.ld_of(zb), false, (int)T.size[r]);  // old nearfield
    }
  }
  g.run(ctx);
  // the new Z replaces the old one; the old arrays return to the contexts'
  // caches, where later work on these streams is ordered after their last use
  Z->mem.swap(nmem);
  Z->mem_aux.swap(naux);
  Z->c = std::move(Zc);
  Z->zero = false;
  step_end(ctx, 7);
}

}  // namespace h2
