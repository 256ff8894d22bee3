// Bases that keep the range of a given matrix exactly and add the truncated
// SVD of what lies outside it: Section 4's leaf case, where range(V_X) is
// kept and the remainder of the induced basis is compressed at eps.  Used by
// phase 1 (the kept matrix is V_X or Vhat_X) and by phase 2 for
// Z <- Z + X Y with Z != 0 (the kept matrix is the old Z's basis).
//
// For each item: K (m x kc) and C (m x nc).
//   1. R factor of K (TSQR), one-sided Jacobi SVD of it: singular values and
//      right vectors V', k1 = #{sigma > 1e-12 sigma_max};
//   2. Householder QR of K V' (columns by descending sigma): its orthogonal
//      factor Q_K has range(K) in its first k1 columns;
//   3. C <- Q_K^* C; the SVD of its rows k1.. (TSQR of their transpose,
//      Jacobi), rank k2 by the truncation rule at eps;
//   4. Q = Q_K [I 0; 0 U2(:, 1:k2)] and [R_K; 0] = Q^* K, R_K = (Q_K^* K)(1:k1, :),
//      the reflectors of step 2 applied to K itself.  (R_Y V'^* equals it only
//      as far as V' is orthogonal: a rank-deficient K leaves V' orthogonal to
//      about the Jacobi tolerance, and that error, carried up through the
//      transfers, would add spurious directions to the parents' kept ranges.)
#include "internal.h"

namespace h2 {

// relative tolerance of the numerical rank of the kept matrix
static constexpr double kKeptRtol = 1e-12;

void kept_compress(h2_ctx* ctx, const std::vector<KeptItem>& items, double eps, Arena& keep, KeptOut& out) {
  const int n = (int)items.size();
  Arena& ws = ctx->ws;  // R_K P (kept by the caller)
  ScopedArena tmp(ctx);  // everything else
  out.k1.assign(n, 0);
  out.k2.assign(n, 0);
  out.Q.assign(n, nullptr);
  out.RKP.assign(n, nullptr);
  if (n == 0) return;
  GemmBatch g, g64;  // g64: plain copies, always in FP64
  g.prec = ctx->prec;
  TsqrBatch ts;
  JacobiBatch jb;
  int32_t* rk = tmp.get<int32_t>(2 * n);  // [k1 | k2] per item
  dev_zero(rk, sizeof(int32_t) * 2 * n, ctx->stream);
  std::vector<double*> Vp(n, nullptr), Yq(n, nullptr), tau(n, nullptr), RYq(n, nullptr), U(n, nullptr);
  std::vector<double*> KQ(n, nullptr);
  // 1. SVD of K from its R factor
  for (int i = 0; i < n; ++i) {
    const KeptItem& it = items[i];
    if (it.m == 0 || it.kc == 0) continue;
    double* Rv = tmp.get<double>((size_t)it.kc * it.kc);
    Vp[i] = tmp.get<double>((size_t)it.kc * it.kc);
    double* sg = tmp.get<double>(it.kc);
    ts.add(it.K, it.ldk, it.m, it.kc, false, Rv, it.kc);
    jb.add(Rv, it.kc, std::min(it.kc, it.m), it.kc, Vp[i], it.kc, sg, rk + i, 0.0, kKeptRtol, nullptr, 1);
  }
  ts.run(ctx);
  jb.run(ctx);
  // 2. Householder QR of K V'
  QrBatch qr;
  for (int i = 0; i < n; ++i) {
    const KeptItem& it = items[i];
    if (!Vp[i]) continue;
    Yq[i] = tmp.get<double>((size_t)it.m * it.kc);
    tau[i] = tmp.get<double>(it.kc);
    RYq[i] = tmp.get<double>((size_t)it.kc * it.kc);
    g.out(Yq[i], it.m, it.m, it.kc);
    g.term(it.K, it.ldk, false, Vp[i], it.kc, false, it.kc);
    qr.add(Yq[i], it.m, it.m, it.kc, tau[i], RYq[i], it.kc, std::min(it.m, it.kc));
    KQ[i] = tmp.get<double>((size_t)it.m * it.kc);  // K, to become Q_K^* K
    g64.out(KQ[i], it.m, it.m, it.kc);
    g64.copy(it.K, it.ldk, false, it.kc);
  }
  g.run(ctx);
  g64.run(ctx);
  qr.run(ctx);
  // 3. remainder: Q_K^* C with the first k1 rows masked, its SVD
  ApplyBatch ap;
  for (int i = 0; i < n; ++i) {
    const KeptItem& it = items[i];
    if (Yq[i] && it.nc > 0) ap.add(Yq[i], it.m, tau[i], it.m, std::min(it.m, it.kc), it.C, it.ldc, it.nc, true);
    if (Yq[i]) ap.add(Yq[i], it.m, tau[i], it.m, std::min(it.m, it.kc), KQ[i], it.m, it.kc, true);
  }
  ap.run(ctx);
  for (int i = 0; i < n; ++i) {
    const KeptItem& it = items[i];
    if (it.m == 0 || it.nc == 0) continue;
    double* Rt = tmp.get<double>((size_t)it.m * it.m);
    U[i] = tmp.get<double>((size_t)it.m * it.m);
    double* sg2 = tmp.get<double>(it.m);
    ts.add(it.C, it.ldc, it.nc, it.m, true, Rt, it.m, 0, rk + i);
    jb.add(Rt, it.m, std::min(it.nc, it.m), it.m, U[i], it.m, sg2, rk + n + i, eps, 0.0, rk + i, 1,
           ctx->rank_rule);
  }
  ts.run(ctx);
  jb.run(ctx);
  const int32_t* kh = read_back(ctx, rk, 2 * n);
  ctx_sync(ctx);
  const std::vector<int32_t> kk(kh, kh + 2 * n);
  // 4. Q = Q_K [I 0; 0 U2], [R_K; 0]
  FillBatch fb;
  for (int i = 0; i < n; ++i) {
    const KeptItem& it = items[i];
    out.k1[i] = kk[i];
    out.k2[i] = kk[n + i];
    const int kt = out.k1[i] + out.k2[i];
    out.Q[i] = keep.get<double>((size_t)std::max(it.m, 1) * std::max(kt, 1));
    fb.add(out.Q[i], std::max(it.m, 1), it.m, kt, 1.0);
  }
  fb.run(ctx);
  for (int i = 0; i < n; ++i) {
    const KeptItem& it = items[i];
    if (out.k2[i] > 0) {
      g64.out(out.Q[i] + (size_t)out.k1[i] * it.m, it.m, it.m, out.k2[i]);
      g64.copy(U[i], it.m, false, out.k2[i]);
    }
  }
  g64.run(ctx);
  for (int i = 0; i < n; ++i) {
    const KeptItem& it = items[i];
    const int kt = out.k1[i] + out.k2[i];
    if (Yq[i] && kt > 0) ap.add(Yq[i], it.m, tau[i], it.m, std::min(it.m, it.kc), out.Q[i], it.m, kt, false);
  }
  ap.run(ctx);
  for (int i = 0; i < n; ++i) {
    const KeptItem& it = items[i];
    const int kt = out.k1[i] + out.k2[i], k1 = out.k1[i];
    out.RKP[i] = ws.get<double>((size_t)std::max(kt, 1) * std::max(it.kc, 1));
    if (kt == 0 || it.kc == 0) continue;
    if (k1 > 0) {  // rows 0..k1-1 of Q_K^* K
      g64.out(out.RKP[i], kt, k1, it.kc);
      g64.copy(KQ[i], it.m, false, it.kc);
    }
    if (kt > k1) g64.out(out.RKP[i] + k1, kt, kt - k1, it.kc);  // zero rows below R_K
  }
  g64.run(ctx);
}

}  // namespace h2
