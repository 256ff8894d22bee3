// Host driver of the symbolic layer (cluster tree, block tree, product tree
// T^XY of Section 6) for sanitizer builds: it links only tree.cpp and no
// device code.  Usage:
//   symbolic_driver <points.f64> <n> <dim> <leaf> <eta> <out.i64>
// reads n x dim points (row-major float64), builds the trees, builds the
// product tree of X Y and of Y^* X^* (transposed views, as the column pass
// does) and writes int64 arrays to <out.i64>, each as (length, values...):
//   perm, off, size, block t, block s, block type,
//   and for each of the two product trees: t, s, type, tri_ptr, tri (4 per
//   triple: s, bx, by, kind), kind_cnt.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../paper_2309_09061_amd/csrc/internal.h"

namespace h2 {
[[noreturn]] void fail(h2_status c, const std::string& msg) { throw Error(c, msg); }
}  // namespace h2

static void put(std::FILE* f, const std::vector<int64_t>& v) {
  const int64_t n = (int64_t)v.size();
  std::fwrite(&n, sizeof n, 1, f);
  if (n) std::fwrite(v.data(), sizeof(int64_t), v.size(), f);
}
template <class V>
static std::vector<int64_t> widen(const V& v) {
  return std::vector<int64_t>(v.begin(), v.end());
}

int main(int argc, char** argv) {
  if (argc != 7) {
    std::fprintf(stderr, "usage: %s points n dim leaf eta out\n", argv[0]);
    return 2;
  }
  const int64_t n = std::atoll(argv[2]);
  const int dim = std::atoi(argv[3]), leaf = std::atoi(argv[4]);
  const double eta = std::atof(argv[5]);
  std::vector<double> pts((size_t)n * dim);
  std::FILE* in = std::fopen(argv[1], "rb");
  if (!in || std::fread(pts.data(), sizeof(double), pts.size(), in) != pts.size()) {
    std::fprintf(stderr, "cannot read points\n");
    return 2;
  }
  std::fclose(in);
  try {
    auto T = h2::build_cluster_tree(dim, n, pts.data(), leaf);
    auto B = h2::build_block_tree(*T, *T, eta);
    h2::H2Core X;
    X.ct = T;
    X.bt = B;
    std::FILE* out = std::fopen(argv[6], "wb");
    put(out, widen(T->perm));
    put(out, widen(T->off));
    put(out, widen(T->size));
    put(out, widen(B->t));
    put(out, widen(B->s));
    put(out, widen(B->type));
    for (int transposed = 0; transposed < 2; ++transposed) {
      h2::View vx{&X, transposed != 0}, vy{&X, transposed != 0};
      const h2::ProductTreeH P = h2::build_product_tree(vx, vy, T->ncl);
      put(out, widen(P.bt->t));
      put(out, widen(P.bt->s));
      put(out, widen(P.bt->type));
      put(out, widen(P.tri_ptr));
      std::vector<int64_t> tri;
      tri.reserve(4 * P.tri.size());
      for (const h2::Triple& q : P.tri) {
        tri.push_back(q.s);
        tri.push_back(q.bx);
        tri.push_back(q.by);
        tri.push_back(q.kind);
      }
      put(out, tri);
      put(out, widen(P.kind_cnt));
    }
    std::fclose(out);
  } catch (const h2::Error& e) {
    std::fprintf(stderr, "h2 error %d: %s\n", (int)e.code, e.what());
    return 1;
  }
  return 0;
}
