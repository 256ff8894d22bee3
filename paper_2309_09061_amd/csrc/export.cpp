// h2_stats and h2_export: sizes and ranks of a handle, and a dump of all of
// its arrays into an uncompressed .npz archive (a zip of .npy files) that
// numpy.load reads.
#include <cstdio>
#include <cstring>

#include "internal.h"

namespace h2 {

namespace {

uint32_t crc32(const uint8_t* p, size_t n, uint32_t crc = 0) {
  static uint32_t table[256];
  static bool init = false;
  if (!init) {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t c = i;
      for (int k = 0; k < 8; ++k) c = (c & 1) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
      table[i] = c;
    }
    init = true;
  }
  crc = ~crc;
  for (size_t i = 0; i < n; ++i) crc = table[(crc ^ p[i]) & 0xFF] ^ (crc >> 8);
  return ~crc;
}

// One array of an archive: a complete .npy file (header + little-endian data).
struct Npy {
  std::string name;
  std::vector<uint8_t> bytes;
};

Npy make_npy(const std::string& name, const char* descr, const std::vector<int64_t>& shape, const void* data,
             size_t nbytes) {
  std::string dict = std::string("{'descr': '") + descr + "', 'fortran_order': False, 'shape': (";
  for (size_t i = 0; i < shape.size(); ++i) dict += std::to_string(shape[i]) + (shape.size() == 1 ? "," : i + 1 < shape.size() ? ", " : "");
  dict += "), }";
  // magic (6) + version (2) + header length (2) + header, padded to 64 with '\n' last
  size_t total = 10 + dict.size() + 1;
  size_t pad = (64 - total % 64) % 64;
  dict += std::string(pad, ' ') + "\n";
  Npy a;
  a.name = name + ".npy";
  a.bytes.reserve(10 + dict.size() + nbytes);
  const uint8_t magic[8] = {0x93, 'N', 'U', 'M', 'P', 'Y', 1, 0};
  a.bytes.insert(a.bytes.end(), magic, magic + 8);
  const uint16_t hl = (uint16_t)dict.size();
  a.bytes.push_back(hl & 0xFF);
  a.bytes.push_back(hl >> 8);
  a.bytes.insert(a.bytes.end(), dict.begin(), dict.end());
  const uint8_t* d = (const uint8_t*)data;
  if (nbytes) a.bytes.insert(a.bytes.end(), d, d + nbytes);
  return a;
}

template <class T>
Npy npy_vec(const std::string& name, const char* descr, const std::vector<T>& v) {
  return make_npy(name, descr, {(int64_t)v.size()}, v.data(), v.size() * sizeof(T));
}

void put16(std::vector<uint8_t>& o, uint16_t v) {
  o.push_back(v & 0xFF);
  o.push_back(v >> 8);
}
void put32(std::vector<uint8_t>& o, uint32_t v) {
  for (int i = 0; i < 4; ++i) o.push_back((v >> (8 * i)) & 0xFF);
}

// Zip archive with stored (uncompressed) members; archives beyond 4 GiB or
// 65535 members are refused (no ZIP64 records are written).
void write_zip(const std::string& path, const std::vector<Npy>& files) {
  FILE* f = std::fopen(path.c_str(), "wb");
  H2_REQUIRE(f, H2_ERR_ARG, "cannot open " + path + " for writing");
  std::vector<uint8_t> central;
  uint64_t off = 0;
  bool ok = files.size() < 0xFFFF;
  for (const Npy& a : files) {
    if (!ok) break;
    if (off + a.bytes.size() + 64 + a.name.size() >= 0xFFFFFFFFull) {
      ok = false;
      break;
    }
    const uint32_t crc = crc32(a.bytes.data(), a.bytes.size());
    std::vector<uint8_t> h;
    put32(h, 0x04034b50);
    put16(h, 20);
    put16(h, 0);
    put16(h, 0);  // stored
    put16(h, 0);
    put16(h, 0x21);  // 1980-01-01
    put32(h, crc);
    put32(h, (uint32_t)a.bytes.size());
    put32(h, (uint32_t)a.bytes.size());
    put16(h, (uint16_t)a.name.size());
    put16(h, 0);
    h.insert(h.end(), a.name.begin(), a.name.end());
    ok = ok && std::fwrite(h.data(), 1, h.size(), f) == h.size();
    ok = ok && (a.bytes.empty() || std::fwrite(a.bytes.data(), 1, a.bytes.size(), f) == a.bytes.size());
    put32(central, 0x02014b50);
    put16(central, 20);
    put16(central, 20);
    put16(central, 0);
    put16(central, 0);
    put16(central, 0);
    put16(central, 0x21);
    put32(central, crc);
    put32(central, (uint32_t)a.bytes.size());
    put32(central, (uint32_t)a.bytes.size());
    put16(central, (uint16_t)a.name.size());
    put16(central, 0);
    put16(central, 0);
    put16(central, 0);
    put16(central, 0);
    put32(central, 0);
    put32(central, (uint32_t)off);
    central.insert(central.end(), a.name.begin(), a.name.end());
    off += h.size() + a.bytes.size();
  }
  std::vector<uint8_t> end;
  put32(end, 0x06054b50);
  put16(end, 0);
  put16(end, 0);
  put16(end, (uint16_t)files.size());
  put16(end, (uint16_t)files.size());
  put32(end, (uint32_t)central.size());
  put32(end, (uint32_t)off);
  put16(end, 0);
  ok = ok && std::fwrite(central.data(), 1, central.size(), f) == central.size();
  ok = ok && std::fwrite(end.data(), 1, end.size(), f) == end.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) {
    std::remove(path.c_str());
    fail(H2_ERR_ARG, "writing " + path + " failed (or the archive would exceed 4 GiB / 65535 members)");
  }
}

// rows x cols column-major matrix at device address p with leading dimension
// ld, appended densely (ld = rows) to out; a NULL p appends zeros
void pull_matrix(h2_ctx* ctx, const double* p, int64_t ld, int64_t rows, int64_t cols, std::vector<double>& out) {
  const size_t base = out.size();
  out.resize(base + (size_t)(rows * cols), 0.0);
  if (!p || rows == 0 || cols == 0) return;
  std::vector<double> tmp((size_t)(ld * (cols - 1) + rows));
  dev_d2h(tmp.data(), p, tmp.size() * sizeof(double), ctx->stream);
  dev_sync(ctx->stream);
  for (int64_t j = 0; j < cols; ++j)
    std::memcpy(out.data() + base + j * rows, tmp.data() + j * ld, rows * sizeof(double));
}

void add_basis(h2_ctx* ctx, const TreeH& T, const Basis& B, const std::string& tag, std::vector<Npy>& files) {
  std::vector<double> leaf, tr;
  std::vector<int64_t> leaf_off(T.ncl + 1, 0), tr_off(T.ncl + 1, 0);
  for (int c = 0; c < T.ncl; ++c) {
    if (T.leaf(c)) pull_matrix(ctx, B.leaf[c], B.leaf_ld[c], T.size[c], B.rank[c], leaf);
    leaf_off[c + 1] = (int64_t)leaf.size();
    if (c > 0) pull_matrix(ctx, B.tr[c], B.tr_ld[c], B.rank[c], B.rank[TreeH::parent(c)], tr);
    tr_off[c + 1] = (int64_t)tr.size();
  }
  files.push_back(npy_vec("rank_" + tag, "<i4", B.rank));
  files.push_back(npy_vec(tag + "_leaf", "<f8", leaf));
  files.push_back(npy_vec(tag + "_leaf_off", "<i8", leaf_off));
  files.push_back(npy_vec(tag + "_transfer", "<f8", tr));
  files.push_back(npy_vec(tag + "_transfer_off", "<i8", tr_off));
}

void add_tree(const TreeH& T, const BlockTreeH& B, std::vector<Npy>& files) {
  files.push_back(npy_vec("perm", "<i8", T.perm));
  files.push_back(npy_vec("cl_off", "<i8", T.off));
  files.push_back(npy_vec("cl_size", "<i8", T.size));
  files.push_back(make_npy("points", "<f8", {T.n, T.dim}, T.pts.data(), T.pts.size() * sizeof(double)));
  files.push_back(npy_vec("blk_row", "<i4", B.t));
  files.push_back(npy_vec("blk_col", "<i4", B.s));
  files.push_back(npy_vec("blk_type", "|i1", B.type));
}

void add_core(h2_ctx* ctx, const H2Core& C, std::vector<Npy>& files) {
  const TreeH& T = *C.ct;
  const BlockTreeH& B = *C.bt;
  add_tree(T, B, files);
  add_basis(ctx, T, C.V, "row", files);
  add_basis(ctx, T, C.W, "col", files);
  std::vector<double> data;
  std::vector<int64_t> off(B.nblocks() + 1, 0);
  for (int b = 0; b < B.nblocks(); ++b) {
    if (B.type[b] == BT_ADM)
      pull_matrix(ctx, C.blk[b], C.ld_of(b), C.V.rank[B.t[b]], C.W.rank[B.s[b]], data);
    else if (B.type[b] == BT_INADM)
      pull_matrix(ctx, C.blk[b], C.ld_of(b), T.size[B.t[b]], T.size[B.s[b]], data);
    off[b + 1] = (int64_t)data.size();
  }
  files.push_back(npy_vec("blk_data", "<f8", data));
  files.push_back(npy_vec("blk_off", "<i8", off));
}

}  // namespace

void export_handle(h2_ctx* ctx, const void* handle, int kind, const std::string& path) {
  std::vector<Npy> files;
  const int32_t k32 = kind;
  files.push_back(make_npy("kind", "<i4", {1}, &k32, sizeof(k32)));
  if (kind == H2_HANDLE_TREE) {
    const h2_tree* t = (const h2_tree*)handle;
    add_tree(*t->ct, *t->bt, files);
  } else if (kind == H2_HANDLE_MATRIX) {
    add_core(ctx, ((const h2_matrix*)handle)->c, files);
  } else {
    add_core(ctx, ((const h2_product*)handle)->c, files);
  }
  write_zip(path, files);
}

void handle_stats(const void* handle, int kind, h2_stats_t* out) {
  std::memset(out, 0, sizeof(*out));
  const TreeH* T = nullptr;
  const BlockTreeH* B = nullptr;
  const H2Core* C = nullptr;
  if (kind == H2_HANDLE_TREE) {
    const h2_tree* t = (const h2_tree*)handle;
    T = t->ct.get();
    B = t->bt.get();
  } else if (kind == H2_HANDLE_MATRIX) {
    const h2_matrix* m = (const h2_matrix*)handle;
    C = &m->c;
    out->device_bytes = (int64_t)(m->mem.total + m->mem_aux.total);
  } else {
    const h2_product* g = (const h2_product*)handle;
    C = &g->c;
    out->device_bytes = (int64_t)(g->mem.total + g->mem_aux.total + g->mem_nf.total);
    out->triples = g->n_triples;
  }
  if (C) {
    T = C->ct.get();
    B = C->bt.get();
  }
  out->n = T->n;
  out->dim = T->dim;
  out->depth = T->depth;
  out->nclusters = T->ncl;
  out->nblocks = B->nblocks();
  out->nadm = B->n_adm;
  out->ninadm = B->n_inadm;
  if (!C) return;
  for (int b = 0; b < B->nblocks(); ++b) {
    if (B->type[b] == BT_ADM)
      out->coupling_entries += (int64_t)C->V.rank[B->t[b]] * C->W.rank[B->s[b]];
    else if (B->type[b] == BT_INADM)
      out->nearfield_entries += T->size[B->t[b]] * T->size[B->s[b]];
  }
  const Basis* bs[2] = {&C->V, &C->W};
  for (int w = 0; w < 2; ++w) {
    int64_t sum = 0;
    for (int l = 0; l <= T->depth && l < H2_STATS_MAX_LEVELS; ++l) {
      int64_t ls = 0;
      int32_t lm = 0;
      for (int c = TreeH::first(l); c < TreeH::first(l + 1); ++c) {
        ls += bs[w]->rank[c];
        lm = std::max(lm, bs[w]->rank[c]);
      }
      out->level_rank_max[w][l] = lm;
      out->level_rank_mean[w][l] = (double)ls / (double)(TreeH::first(l + 1) - TreeH::first(l));
      out->rank_max[w] = std::max(out->rank_max[w], lm);
      sum += ls;
    }
    out->rank_mean[w] = (double)sum / (double)T->ncl;
  }
}

}  // namespace h2
