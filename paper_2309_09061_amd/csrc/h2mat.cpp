// H^2-matrices on the device: construction by Chebyshev interpolation
// (Section 2, Example "Integral operator"), zero matrices, the O(nk)
// matrix-vector product (forward transform, couplings, backward transform,
// nearfield) and densification for tests.
#include <cmath>

#include "internal.h"

namespace h2 {

void compress_kernel(h2_ctx* ctx, const h2_tree* tree, int kernel, int order, const double* normals,
                     h2_matrix* out) {
  const TreeH& T = *tree->ct;
  const BlockTreeH& B = *tree->bt;
  int k = 1;
  for (int a = 0; a < T.dim; ++a) k *= order;
  H2_REQUIRE(order >= 1 && k <= 128, H2_ERR_ARG, "order^dim must be in [1, 128]");
  const bool dlp = kernel == H2_K_DLP;
  H2_REQUIRE(!dlp || normals, H2_ERR_ARG, "the double-layer kernel needs the normals at the points");
  out->ctx = ctx;
  out->mem.bind(ctx);
  H2Core& C = out->c;
  C.ct = tree->ct;
  C.bt = tree->bt;
  C.V.resize(T.ncl);
  Arena& A = out->mem;
  // Interpolation boxes: the (widened) cluster boxes; for the double-layer
  // kernel their bounding cubes (same center, every edge the longest one),
  // since a cluster on one face of a surface has a flat box on which the
  // derivative across the face would be determined by rounding
  std::vector<double> blo = T.lo, bhi = T.hi;
  if (dlp)
    for (int c = 0; c < T.ncl; ++c) {
      double* l = &blo[(size_t)c * T.dim];
      double* h = &bhi[(size_t)c * T.dim];
      double edge = 0.0;
      for (int a = 0; a < T.dim; ++a) edge = std::max(edge, h[a] - l[a]);
      const double half = 0.5 * edge;
      for (int a = 0; a < T.dim; ++a) {
        const double mid = 0.5 * (l[a] + h[a]);
        l[a] = mid - half;
        h[a] = mid + half;
      }
    }
  // geometry on the device (points and normals in cluster order)
  double* pts = A.get<double>(T.pts.size());
  double* lo = A.get<double>(blo.size());
  double* hi = A.get<double>(bhi.size());
  dev_h2d(pts, T.pts.data(), T.pts.size() * 8, ctx->stream);
  dev_h2d(lo, blo.data(), blo.size() * 8, ctx->stream);
  dev_h2d(hi, bhi.data(), bhi.size() * 8, ctx->stream);
  double* nrm = nullptr;
  if (dlp) {
    std::vector<double> nc((size_t)T.n * T.dim);
    for (int64_t p = 0; p < T.n; ++p)
      for (int a = 0; a < T.dim; ++a) {
        const double v = normals[T.perm[p] * T.dim + a];
        H2_REQUIRE(std::isfinite(v), H2_ERR_NUMERIC, "non-finite normal");
        nc[(size_t)p * T.dim + a] = v;
      }
    nrm = A.get<double>(nc.size());
    dev_h2d(nrm, nc.data(), nc.size() * 8, ctx->stream);
    dev_sync(ctx->stream);  // nc is a host temporary
  }
  // leaf bases and transfers (the column basis of the double-layer kernel
  // has plain interpolation leaves and the row basis's transfers)
  std::vector<ChebLeaf> leaves, wleaves;
  std::vector<ChebPair> transfers;
  Basis Wb;
  if (dlp) Wb.resize(T.ncl);
  for (int c = 0; c < T.ncl; ++c) {
    C.V.rank[c] = k;
    if (T.leaf(c)) {
      double* V = A.get<double>((size_t)T.size[c] * k);
      C.V.leaf[c] = V;
      C.V.leaf_ld[c] = std::max<int64_t>(T.size[c], 1);
      leaves.push_back({V, C.V.leaf_ld[c], T.off[c], c, (int32_t)T.size[c]});
      if (dlp) {
        double* Wl = A.get<double>((size_t)T.size[c] * k);
        Wb.leaf[c] = Wl;
        Wb.leaf_ld[c] = C.V.leaf_ld[c];
        wleaves.push_back({Wl, Wb.leaf_ld[c], T.off[c], c, (int32_t)T.size[c]});
      }
    }
    if (c > 0) {
      double* E = A.get<double>((size_t)k * k);
      C.V.tr[c] = E;
      C.V.tr_ld[c] = k;
      transfers.push_back({E, k, c, TreeH::parent(c)});
    }
  }
  // couplings and nearfield
  C.blk.assign(B.nblocks(), nullptr);
  std::vector<ChebPair> coup;
  std::vector<NearBlock> near;
  for (int b = 0; b < B.nblocks(); ++b) {
    if (B.type[b] == BT_ADM) {
      double* S = A.get<double>((size_t)k * k);
      C.blk[b] = S;
      coup.push_back({S, k, B.t[b], B.s[b]});
    } else if (B.type[b] == BT_INADM) {
      int64_t mt = T.size[B.t[b]], ms = T.size[B.s[b]];
      double* N = A.get<double>((size_t)mt * ms);
      C.blk[b] = N;
      near.push_back({N, std::max<int64_t>(mt, 1), T.off[B.t[b]], T.off[B.s[b]], (int32_t)mt, (int32_t)ms,
                      B.t[b] == B.s[b] ? 1 : 0, 0});
    }
  }
  if (dlp) {
    // <n(x), x - y>/(4 pi |x - y|^3) = -<n(x), grad_x gamma(x, y)> with
    // gamma = 1/(4 pi |x - y|): interpolate gamma, differentiate the row side
    for (int c = 0; c < T.ncl; ++c) {
      Wb.rank[c] = k;
      Wb.tr[c] = C.V.tr[c];
      Wb.tr_ld[c] = C.V.tr_ld[c];
    }
    C.W = Wb;
    k_cheb_leaf_dn(upload(ctx, leaves), (int)leaves.size(), pts, nrm, lo, hi, T.dim, order, ctx->stream);
    k_cheb_leaf(upload(ctx, wleaves), (int)wleaves.size(), pts, lo, hi, T.dim, order, ctx->stream);
  } else {
    C.W = C.V;  // the same interpolation on both sides
    k_cheb_leaf(upload(ctx, leaves), (int)leaves.size(), pts, lo, hi, T.dim, order, ctx->stream);
  }
  k_cheb_transfer(upload(ctx, transfers), (int)transfers.size(), lo, hi, T.dim, order, ctx->stream);
  k_cheb_coupling(upload(ctx, coup), (int)coup.size(), lo, hi, T.dim, order, dlp ? H2_K_INV4PI : kernel,
                  ctx->stream);
  k_nearfield(upload(ctx, near), (int)near.size(), pts, nrm, T.dim, kernel, ctx->stream);
}

void zero_like(h2_ctx* ctx, const h2_tree* tree, double eta_Z, h2_matrix* out) {
  out->ctx = ctx;
  out->mem.bind(ctx);
  out->zero = true;
  out->c.ct = tree->ct;
  out->c.bt = eta_Z > 0 && eta_Z != tree->eta ? build_block_tree(*tree->ct, *tree->ct, eta_Z) : tree->bt;
  out->c.V.resize(tree->ct->ncl);
  out->c.W.resize(tree->ct->ncl);
  out->c.blk.assign(tree->bt->nblocks(), nullptr);
}

// full cluster basis matrices (#c x rank c, ld #c) for every cluster
static std::vector<double*> full_basis(h2_ctx* ctx, const TreeH& T, const Basis& V) {
  std::vector<double*> F(T.ncl, nullptr);
  for (int c = 0; c < T.ncl; ++c) F[c] = ctx->ws.get<double>((size_t)T.size[c] * std::max(V.rank[c], 1));
  GemmBatch g;
  for (int c = T.first(T.depth); c < T.ncl; ++c) {
    g.out(F[c], T.size[c], (int)T.size[c], V.rank[c]);
    g.copy(V.leaf[c], V.leaf_ld[c], false, V.rank[c]);
  }
  g.run(ctx);
  for (int l = T.depth - 1; l >= 0; --l) {
    for (int c = T.first(l); c < T.first(l + 1); ++c)
      for (int q = 1; q <= 2; ++q) {
        int ch = 2 * c + q;
        g.out(F[c] + (T.off[ch] - T.off[c]), T.size[c], (int)T.size[ch], V.rank[c]);
        g.term(F[ch], T.size[ch], false, V.tr[ch], V.tr_ld[ch], false, V.rank[ch]);
      }
    g.run(ctx);
  }
  return F;
}

void basis_dense(h2_ctx* ctx, const H2Core& A, int which, int cluster, double* out, int64_t ld) {
  const TreeH& T = *A.ct;
  const Basis& V = which == 0 ? A.V : A.W;
  H2_REQUIRE(cluster >= 0 && cluster < T.ncl, H2_ERR_ARG, "cluster out of range");
  H2_REQUIRE(ld >= T.size[cluster], H2_ERR_ARG, "ld too small");
  auto F = full_basis(ctx, T, V);
  GemmBatch g;
  g.out(out, ld, (int)T.size[cluster], V.rank[cluster]);
  g.copy(F[cluster], T.size[cluster], false, V.rank[cluster]);
  g.run(ctx);
}

void to_dense(h2_ctx* ctx, const H2Core& A, double* out, int64_t ld) {
  const TreeH& T = *A.ct;
  const BlockTreeH& B = *A.bt;
  auto Vf = full_basis(ctx, T, A.V);
  auto Wf = full_basis(ctx, T, A.W);
  GemmBatch g1, g2;
  std::vector<double*> tmp(B.nblocks(), nullptr);
  for (int b = 0; b < B.nblocks(); ++b) {
    int t = B.t[b], s = B.s[b];
    double* O = out + T.off[t] + T.off[s] * ld;
    if (B.type[b] == BT_ADM) {
      int kt = A.V.rank[t], ks = A.W.rank[s];
      if (kt == 0 || ks == 0 || !A.blk[b]) {
        g2.out(O, ld, (int)T.size[t], (int)T.size[s]);  // zero
        continue;
      }
      tmp[b] = ctx->ws.get<double>((size_t)kt * T.size[s]);
      g1.out(tmp[b], kt, kt, (int)T.size[s]);
      g1.term(A.blk[b], A.ld_of(b), false, Wf[s], T.size[s], true, ks);
      g2.out(O, ld, (int)T.size[t], (int)T.size[s]);
      g2.term(Vf[t], T.size[t], false, tmp[b], kt, false, kt);
    } else if (B.type[b] == BT_INADM) {
      g2.out(O, ld, (int)T.size[t], (int)T.size[s]);
      if (A.blk[b]) g2.copy(A.blk[b], A.ld_of(b), false, (int)T.size[s]);
    }
  }
  g1.run(ctx);
  g2.run(ctx);
}

// z = op(A) x (z n x nvec, ld n), then y = alpha z + beta y
void matvec(h2_ctx* ctx, const H2Core& A, bool trans, double alpha, const double* x, double beta,
            double* y, int nvec) {
  const TreeH& T = *A.ct;
  View v{&A, trans};
  const Basis& R = v.rowb();
  const Basis& Cb = v.colb();
  int64_t n = T.n;
  std::vector<double*> xh(T.ncl), yh(T.ncl);
  for (int c = 0; c < T.ncl; ++c) {
    xh[c] = ctx->ws.get<double>((size_t)std::max(Cb.rank[c], 1) * nvec);
    yh[c] = ctx->ws.get<double>((size_t)std::max(R.rank[c], 1) * nvec);
  }
  GemmBatch g;
  // forward transform
  for (int c = T.first(T.depth); c < T.ncl; ++c) {
    g.out(xh[c], Cb.rank[c], Cb.rank[c], nvec);
    g.term(Cb.leaf[c], Cb.leaf_ld[c], true, x + T.off[c], n, false, (int)T.size[c]);
  }
  g.run(ctx);
  for (int l = T.depth - 1; l >= 0; --l) {
    for (int c = T.first(l); c < T.first(l + 1); ++c) {
      g.out(xh[c], Cb.rank[c], Cb.rank[c], nvec);
      for (int q = 1; q <= 2; ++q) {
        int ch = 2 * c + q;
        g.term(Cb.tr[ch], Cb.tr_ld[ch], true, xh[ch], Cb.rank[ch], false, Cb.rank[ch]);
      }
    }
    g.run(ctx);
  }
  // couplings
  for (int t = 0; t < T.ncl; ++t) {
    g.out(yh[t], R.rank[t], R.rank[t], nvec);
    const int32_t* bl;
    int cnt;
    v.row_blocks(t, bl, cnt);
    for (int q = 0; q < cnt; ++q) {
      int b = bl[q];
      if (v.type(b) != BT_ADM || !v.ptr(b)) continue;
      int s = v.vcol(b);
      g.term(v.ptr(b), v.ld(b), trans, xh[s], Cb.rank[s], false, Cb.rank[s]);
    }
  }
  g.run(ctx);
  // backward transform
  for (int l = 1; l <= T.depth; ++l) {
    for (int c = T.first(l); c < T.first(l + 1); ++c) {
      g.out(yh[c], R.rank[c], R.rank[c], nvec, true);
      g.term(R.tr[c], R.tr_ld[c], false, yh[TreeH::parent(c)], R.rank[TreeH::parent(c)], false,
             R.rank[TreeH::parent(c)]);
    }
    g.run(ctx);
  }
  // leaves and nearfield
  double* z = ctx->ws.get<double>((size_t)n * nvec);
  for (int t = T.first(T.depth); t < T.ncl; ++t) {
    g.out(z + T.off[t], n, (int)T.size[t], nvec);
    g.term(R.leaf[t], R.leaf_ld[t], false, yh[t], R.rank[t], false, R.rank[t]);
    const int32_t* bl;
    int cnt;
    v.row_blocks(t, bl, cnt);
    for (int q = 0; q < cnt; ++q) {
      int b = bl[q];
      if (v.type(b) != BT_INADM || !v.ptr(b)) continue;
      int s = v.vcol(b);
      g.term(v.ptr(b), v.ld(b), trans, x + T.off[s], n, false, (int)T.size[s]);
    }
  }
  g.run(ctx);
  k_axpby(n, nvec, alpha, z, n, beta, y, n, ctx->stream);
}

}  // namespace h2
