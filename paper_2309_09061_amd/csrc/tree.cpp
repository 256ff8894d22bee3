// Cluster trees, block trees and the product block tree T^XY (host, integer
// work).  Section 2: Definitions "Cluster tree" and "Block tree"; Section 6:
// the product block tree and its admissible / inadmissible leaves.
#include <algorithm>
#include <cmath>
#include <exception>
#include <numeric>
#include <thread>

#include "internal.h"

namespace h2 {

// Median bisection along the longest edge of the tight bounding box (lowest
// axis on ties), points ordered by (coordinate, original index); the first
// floor(m/2) points form child 2c+1.  All branches reach the common depth
// D = min{D >= 0 : leaf_size 2^D >= n}, so every leaf lies on level D.
std::shared_ptr<TreeH> build_cluster_tree(int dim, int64_t n, const double* pts, int leaf_size) {
  H2_REQUIRE(dim >= 1 && dim <= 3, H2_ERR_ARG, "dim must be 1, 2 or 3");
  H2_REQUIRE(n >= 1, H2_ERR_ARG, "n must be positive");
  H2_REQUIRE(leaf_size >= 2, H2_ERR_ARG, "leaf_size must be >= 2");
  for (int64_t i = 0; i < n * dim; ++i)
    H2_REQUIRE(std::isfinite(pts[i]), H2_ERR_NUMERIC, "non-finite point coordinate");
  auto T = std::make_shared<TreeH>();
  T->dim = dim;
  T->n = n;
  int depth = 0;
  while ((int64_t)leaf_size << depth < n) ++depth;
  H2_REQUIRE(depth <= 24, H2_ERR_ARG, "tree too deep");
  T->depth = depth;
  int ncl = (2 << depth) - 1;
  T->ncl = ncl;
  T->off.assign(ncl, 0);
  T->size.assign(ncl, 0);
  T->blo.assign((size_t)ncl * dim, 0);
  T->bhi.assign((size_t)ncl * dim, 0);
  std::vector<int64_t> idx(n);
  std::iota(idx.begin(), idx.end(), 0);
  // every cluster is a contiguous range of idx; children ranges stay contiguous
  T->off[0] = 0;
  T->size[0] = n;
  for (int c = 0; c < ncl; ++c) {
    int64_t o = T->off[c], m = T->size[c];
    double* lo = &T->blo[(size_t)c * dim];
    double* hi = &T->bhi[(size_t)c * dim];
    for (int a = 0; a < dim; ++a) {
      lo[a] = INFINITY;
      hi[a] = -INFINITY;
    }
    for (int64_t q = 0; q < m; ++q) {
      const double* p = pts + idx[o + q] * dim;
      for (int a = 0; a < dim; ++a) {
        lo[a] = std::min(lo[a], p[a]);
        hi[a] = std::max(hi[a], p[a]);
      }
    }
    if (TreeH::level(c) < depth) {
      int ax = 0;
      double best = hi[0] - lo[0];
      for (int a = 1; a < dim; ++a)
        if (hi[a] - lo[a] > best) {
          best = hi[a] - lo[a];
          ax = a;
        }
      std::sort(idx.begin() + o, idx.begin() + o + m, [&](int64_t i, int64_t j) {
        double xi = pts[i * dim + ax], xj = pts[j * dim + ax];
        return xi < xj || (xi == xj && i < j);
      });
      int64_t h = m / 2;
      T->off[2 * c + 1] = o;
      T->size[2 * c + 1] = h;
      T->off[2 * c + 2] = o + h;
      T->size[2 * c + 2] = m - h;
    }
  }
  T->perm = idx;
  T->pts.resize((size_t)n * dim);
  for (int64_t p = 0; p < n; ++p)
    for (int a = 0; a < dim; ++a) T->pts[(size_t)p * dim + a] = pts[idx[p] * dim + a];
  // interpolation boxes: edges narrower than 1e-12 diam(root) are widened
  double d0 = 0;
  for (int a = 0; a < dim; ++a) {
    double w = T->bhi[a] - T->blo[a];
    d0 += w * w;
  }
  double floor_w = 1e-12 * std::sqrt(d0);
  T->lo = T->blo;
  T->hi = T->bhi;
  for (int c = 0; c < ncl; ++c)
    for (int a = 0; a < dim; ++a) {
      double& l = T->lo[(size_t)c * dim + a];
      double& h = T->hi[(size_t)c * dim + a];
      if (h - l < floor_w) {
        double mid = 0.5 * (l + h);
        l = mid - 0.5 * floor_w;
        h = mid + 0.5 * floor_w;
      }
    }
  return T;
}

static double box_diam(const TreeH& T, int c) {
  double s = 0;
  for (int a = 0; a < T.dim; ++a) {
    double w = T.bhi[(size_t)c * T.dim + a] - T.blo[(size_t)c * T.dim + a];
    s += w * w;
  }
  return std::sqrt(s);
}

static double box_dist(const TreeH& A, int a, const TreeH& B, int b) {
  double s = 0;
  for (int q = 0; q < A.dim; ++q) {
    double g1 = B.blo[(size_t)b * A.dim + q] - A.bhi[(size_t)a * A.dim + q];
    double g2 = A.blo[(size_t)a * A.dim + q] - B.bhi[(size_t)b * A.dim + q];
    double g = std::max(0.0, std::max(g1, g2));
    s += g * g;
  }
  return std::sqrt(s);
}

void BlockTreeH::finalize(int ncl) {
  int nb = nblocks();
  row_ptr.assign(ncl + 1, 0);
  col_ptr.assign(ncl + 1, 0);
  n_adm = n_inadm = 0;
  for (int b = 0; b < nb; ++b) {
    row_ptr[t[b] + 1]++;
    col_ptr[s[b] + 1]++;
    n_adm += type[b] == BT_ADM;
    n_inadm += type[b] == BT_INADM;
  }
  for (int c = 0; c < ncl; ++c) {
    row_ptr[c + 1] += row_ptr[c];
    col_ptr[c + 1] += col_ptr[c];
  }
  row_blk.assign(nb, 0);
  col_blk.assign(nb, 0);
  std::vector<int32_t> rp(row_ptr.begin(), row_ptr.end() - 1), cp(col_ptr.begin(), col_ptr.end() - 1);
  for (int b = 0; b < nb; ++b) {
    row_blk[rp[t[b]]++] = b;
    col_blk[cp[s[b]]++] = b;
  }
  for (int c = 0; c < ncl; ++c) {
    std::sort(row_blk.begin() + row_ptr[c], row_blk.begin() + row_ptr[c + 1],
              [&](int x, int y) { return s[x] < s[y]; });
    std::sort(col_blk.begin() + col_ptr[c], col_blk.begin() + col_ptr[c + 1],
              [&](int x, int y) { return t[x] < t[y]; });
  }
}

int BlockTreeH::find(int tt, int ss) const {
  int lo = row_ptr[tt], hi = row_ptr[tt + 1];
  while (lo < hi) {
    int mid = (lo + hi) / 2;
    int v = s[row_blk[mid]];
    if (v == ss) return row_blk[mid];
    if (v < ss)
      lo = mid + 1;
    else
      hi = mid;
  }
  return -1;
}

// Standard admissibility: dist(t,s) > 0 and max(diam t, diam s) <= eta dist.
// Refinement from (root, root) stops at admissible blocks and leaf x leaf.
std::shared_ptr<BlockTreeH> build_block_tree(const TreeH& rt, const TreeH& ct, double eta) {
  H2_REQUIRE(rt.depth == ct.depth, H2_ERR_SHAPE, "row and column trees differ in depth");
  auto B = std::make_shared<BlockTreeH>();
  B->lvl.push_back(0);
  B->t.push_back(0);
  B->s.push_back(0);
  for (int l = 0; l <= rt.depth; ++l) {
    int b0 = B->lvl[l], b1 = (int)B->t.size();
    for (int b = b0; b < b1; ++b) {
      int tt = B->t[b], ss = B->s[b];
      double dist = box_dist(rt, tt, ct, ss);
      bool adm = dist > 0.0 && std::max(box_diam(rt, tt), box_diam(ct, ss)) <= eta * dist;
      if (adm) {
        B->type.push_back(BT_ADM);
        B->child0.push_back(-1);
      } else if (l == rt.depth) {
        B->type.push_back(BT_INADM);
        B->child0.push_back(-1);
      } else {
        B->type.push_back(BT_SPLIT);
        B->child0.push_back((int)B->t.size());
        for (int a = 1; a <= 2; ++a)
          for (int c = 1; c <= 2; ++c) {
            B->t.push_back(2 * tt + a);
            B->s.push_back(2 * ss + c);
          }
      }
    }
    B->lvl.push_back(b1);
  }
  B->finalize(rt.ncl);
  return B;
}

// T^XY: (t,r) is subdivided iff some middle s has (t,s) and (s,r) both
// subdivided; a leaf is admissible iff every middle s has an admissible
// factor.  The triples (t,s,r) reaching a block are recorded: terminated
// ones with their kind (both factors admissible, only (t,s), only (s,r),
// neither).
// child (a, c) (a: row child, c: column child, 1 or 2, view coordinates) of
// the subdivided block b of a view; block trees list the four children of a
// block row-child-major
static inline int view_child(const int32_t* child0, bool transposed, int b, int a, int c) {
  const int c0 = child0[b];
  return transposed ? c0 + (c - 1) * 2 + (a - 1) : c0 + (a - 1) * 2 + (c - 1);
}

// f(i0, i1) over [0, n) in contiguous parts on up to `threads` host threads,
// split so that the parts hold about equal shares of the weights given by
// the prefix sums w (w[0] = 0, w[n] = total); the first exception is rethrown
template <typename F>
static void parallel_parts(int n, const std::vector<int64_t>& w, int threads, F f) {
  if (threads <= 1 || n < 2 * threads) {
    f(0, n);
    return;
  }
  std::vector<int> cut(threads + 1, n);
  cut[0] = 0;
  for (int p = 1; p < threads; ++p) {
    const int64_t target = w[n] * p / threads;
    cut[p] = (int)(std::lower_bound(w.begin(), w.begin() + n + 1, target) - w.begin());
    cut[p] = std::max(cut[p], cut[p - 1]);
  }
  std::vector<std::exception_ptr> err(threads);
  std::vector<std::thread> th;
  for (int p = 1; p < threads; ++p)
    th.emplace_back([&, p] {
      try {
        f(cut[p], cut[p + 1]);
      } catch (...) {
        err[p] = std::current_exception();
      }
    });
  try {
    f(cut[0], cut[1]);
  } catch (...) {
    err[0] = std::current_exception();
  }
  for (auto& t : th) t.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

// Level by level: the middle triples (s, block of X, block of Y) reaching each
// block of the level (stored flat with offsets) are first counted per block
// (terminated ones, by kind, and subdivided ones), then, with the offsets
// from prefix sums, each block writes its terminated triples, its children
// and their middle triples in place.  Blocks are independent, so both sweeps
// run on several host threads for the wide levels; the result is the same
// as a sequential build.
ProductTreeH build_product_tree(const View& X, const View& Y, int ncl) {
  ProductTreeH P;
  auto B = std::make_shared<BlockTreeH>();
  P.bt = B;
  struct Mid {
    int32_t s, bx, by;
  };
  const int8_t* tyX = X.m->bt->type.data();
  const int8_t* tyY = Y.m->bt->type.data();
  const int32_t* chX = X.m->bt->child0.data();
  const int32_t* chY = Y.m->bt->child0.data();
  const bool trX = X.T, trY = Y.T;
  std::vector<Mid, DefaultInit<Mid>> mids_cur, mids_next;
  std::vector<int64_t> off_cur{0, 1}, off_next;
  {
    const int bx = X.find(0, 0), by = Y.find(0, 0);
    H2_REQUIRE(bx >= 0 && by >= 0, H2_ERR_SHAPE, "product tree: missing root block");
    mids_cur.push_back({0, bx, by});
  }
  B->lvl.push_back(0);
  B->t.push_back(0);
  B->s.push_back(0);
  const int depth = X.m->ct->depth;
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  P.tri_ptr.push_back(0);
  for (int l = 0; l <= depth; ++l) {
    const int b0 = B->lvl[l], b1 = (int)B->t.size(), nb = b1 - b0;
    // two workers: more compete with the passes' host threads (measured: no
    // faster with four or eight)
    const int threads = mids_cur.size() >= 65536 ? std::min(2, hw) : 1;
    // ---- counts per block: terminated triples and subdivided middles ----
    std::vector<int64_t> nterm(nb + 1, 0), nrec(nb + 1, 0);
    parallel_parts(nb, off_cur, threads, [&](int i0, int i1) {
      for (int i = i0; i < i1; ++i) {
        int64_t t = 0, r = 0;
        bool nn = false;
        for (int64_t q = off_cur[i]; q < off_cur[i + 1]; ++q) {
          const int8_t tx = tyX[mids_cur[q].bx], ty = tyY[mids_cur[q].by];
          if (tx == BT_SPLIT && ty == BT_SPLIT) {
            ++r;
            continue;
          }
          if (tx != BT_ADM && ty != BT_ADM) {
            H2_REQUIRE(tx == BT_INADM && ty == BT_INADM, H2_ERR_UNSUPPORTED,
                       "product tree: non-level-aligned factor blocks");
            nn = true;
          }
          ++t;
        }
        H2_REQUIRE(!(nn && r > 0), H2_ERR_UNSUPPORTED, "product tree: dense triple above the leaf level");
        nterm[i] = t;
        nrec[i] = r;
      }
    });
    // ---- offsets ----
    std::vector<int64_t> tri_off(nb + 1), kid_off(nb + 1), mid_off(nb + 1);
    tri_off[0] = kid_off[0] = mid_off[0] = 0;
    for (int i = 0; i < nb; ++i) {
      tri_off[i + 1] = tri_off[i] + nterm[i];
      kid_off[i + 1] = kid_off[i] + (nrec[i] ? 4 : 0);
      mid_off[i + 1] = mid_off[i] + 8 * nrec[i];
    }
    const size_t tri0 = P.tri.size();
    const int nkids = (int)kid_off[nb];
    P.tri.resize(tri0 + tri_off[nb]);
    P.tri_ptr.resize((size_t)b1 + 1);
    P.kind_cnt.resize(4 * (size_t)b1, 0);
    B->type.resize(b1);
    B->child0.resize(b1);
    B->t.resize((size_t)b1 + nkids);
    B->s.resize((size_t)b1 + nkids);
    mids_next.resize(mid_off[nb]);
    off_next.assign((size_t)nkids + 1, 0);
    // ---- fill ----
    parallel_parts(nb, off_cur, threads, [&](int i0, int i1) {
      for (int i = i0; i < i1; ++i) {
        const int b = b0 + i, tt = B->t[b], rr = B->s[b];
        int64_t tp = tri0 + tri_off[i], r = 0;
        bool nn = false;
        const int64_t nr = nrec[i];
        const int kid = b1 + (int)kid_off[i];
        for (int64_t q = off_cur[i]; q < off_cur[i + 1]; ++q) {
          const Mid md = mids_cur[q];
          const int8_t tx = tyX[md.bx], ty = tyY[md.by];
          if (tx == BT_SPLIT && ty == BT_SPLIT) {
            for (int a = 1; a <= 2; ++a)
              for (int c = 1; c <= 2; ++c) {
                const int k = (a - 1) * 2 + (c - 1);
                Mid* dst = &mids_next[mid_off[i] + (int64_t)k * 2 * nr + 2 * r];
                for (int qq = 1; qq <= 2; ++qq)
                  dst[qq - 1] = {2 * md.s + qq, view_child(chX, trX, md.bx, a, qq), view_child(chY, trY, md.by, qq, c)};
              }
            ++r;
            continue;
          }
          int8_t kind;
          if (tx == BT_ADM && ty == BT_ADM)
            kind = TK_AA;
          else if (tx == BT_ADM)
            kind = TK_AN;
          else if (ty == BT_ADM)
            kind = TK_NA;
          else {
            kind = TK_NN;
            nn = true;
          }
          P.tri[tp++] = {md.s, md.bx, md.by, (int32_t)kind};
          P.kind_cnt[4 * (size_t)b + kind]++;
        }
        P.tri_ptr[b + 1] = (int32_t)tp;
        if (nr) {
          B->type[b] = BT_SPLIT;
          B->child0[b] = kid;
          for (int a = 1; a <= 2; ++a)
            for (int c = 1; c <= 2; ++c) {
              const int k = (a - 1) * 2 + (c - 1);
              B->t[kid + k] = 2 * tt + a;
              B->s[kid + k] = 2 * rr + c;
              off_next[kid - b1 + k + 1] = mid_off[i] + (int64_t)(k + 1) * 2 * nr;
            }
        } else {
          B->type[b] = nn ? BT_INADM : BT_ADM;
          B->child0[b] = -1;
        }
      }
    });
    P.n_terminated += tri_off[nb];
    B->lvl.push_back(b1);
    mids_cur.swap(mids_next);
    off_cur.swap(off_next);
  }
  B->finalize(ncl);
  return P;
}

}  // namespace h2
