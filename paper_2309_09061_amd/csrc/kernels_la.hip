// Batched dense linear algebra for gfx950 (CDNA4, 64-lane wavefronts).
//
//  gemm_sum  grouped variable-size products C = beta C + sum alpha op(A) op(B)
//            on FP64 MFMA (v_mfma_f64_16x16x4f64), one wavefront per 16x16
//            output tile, the terms of one output accumulated in registers
//  qr        Householder QR of small matrices, reflectors kept (LAPACK
//            conventions: H = I - tau v v^T, v_j = 1), R copied out
//  apply     C <- Q^T C or Q C with the reflectors of qr
//  tsqr      R factor of tall (or transposed wide) matrices, streamed in row
//            chunks through a stacked [R; chunk] Householder QR
//  jacobi    one-sided (Hestenes) Jacobi SVD with round-robin parallel pair
//            ordering; singular values and right singular vectors of R
//  fill      batched block fill (zeros with a constant diagonal)
//
// Working sets live in LDS (up to the device limit, 160 KiB per workgroup on
// gfx950) and otherwise in a per-workgroup slot of global scratch.  The host
// passes the LDS capacity of each launch; a problem uses LDS iff its working
// set fits that capacity, the same predicate the host used to size it.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <type_traits>

#include "internal.h"

namespace h2 {

typedef double v4d __attribute__((ext_vector_type(4)));

#define HIP_OK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) fail(H2_ERR_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

// Cross-lane sums.  Within a row of 16 lanes DPP moves are used (register
// to register, no LDS round trip): quad_perm [1,0,3,2] and [2,3,0,1] pair
// lanes at distance 1 and 2, row_half_mirror (i <-> 7 - i) joins the two
// quads of each group of 8, row_mirror (i <-> 15 - i) the two halves of each
// row.  Every lane of a group ends with the same, order-independent sum
// because each step adds two equal partial sums in either order.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// sum over aligned groups of g lanes (g a power of two <= 64, uniform); all
// lanes of a group must be active
__device__ __forceinline__ double group_sum(double v, int g) {
  if (g >= 2) v += dpp_move<0xB1>(v);
  if (g >= 4) v += dpp_move<0x4E>(v);
  if (g >= 8) v += dpp_move<0x141>(v);
  if (g >= 16) v += dpp_move<0x140>(v);
  if (g >= 32) v += __shfl_xor(v, 16, 64);
  if (g >= 64) v += __shfl_xor(v, 32, 64);
  return v;
}

__device__ inline double wave_sum(double v) { return group_sum(v, 64); }

// block-wide sum for 256 threads (4 waves); `red` has >= 4 doubles
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
// grouped GEMM on FP64 MFMA
// ---------------------------------------------------------------------------
typedef float v4f __attribute__((ext_vector_type(4)));

typedef short v4s __attribute__((ext_vector_type(4)));

// bfloat16 of a float by round-to-nearest-even (finite values), as its bits
__device__ __forceinline__ short bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(short h) { return __uint_as_float((uint32_t)(uint16_t)h << 16); }

// MFMA steps of a 16 x 16 product in the arithmetic of the bulk products:
//   P = 0  FP64 (v_mfma_f64_16x16x4f64), one k per lane and step;
//   P = 1  FP32: operands rounded to FP32, FP32 accumulation (16x16x4f32);
//   P = 2  BF16 hi/lo: each operand a = a_h + a_l with a_h = bf16(a) and
//          a_l = bf16(a - a_h), and a b ~ a_h b_h + a_h b_l + a_l b_h, three
//          v_mfma_f32_16x16x16_bf16 with FP32 accumulation (about 2^-16
//          relative per product);
//   P = 3  plain BF16: a_h b_h only (about 2^-8 relative).
// A step consumes KG values of k: lane (r, q) holds EPL = KG / 4 of them,
// k = l0 + kof(u, q) for u < EPL (any bijection onto the chunk gives the same
// sum; the BF16 instruction takes four consecutive k per lane).
// Accumulator layouts (measured on gfx950): FP64 register v of lane (r, q)
// holds D[4v + q][r]; FP32 register v holds D[4q + v][r].
template <int P>
struct Mfma16 {
  static constexpr int KG = P >= 2 ? 16 : 4;
  static constexpr int EPL = KG / 4;
  typedef typename std::conditional<P == 0, v4d, v4f>::type acc_t;
  static __device__ __forceinline__ acc_t zero() {
    acc_t z = {0, 0, 0, 0};
    return z;
  }
  static __device__ __forceinline__ int kof(int u, int q) { return P >= 2 ? 4 * q + u : q; }
  static __device__ __forceinline__ acc_t step(const double* a, const double* b, acc_t c) {
    if constexpr (P == 0) {
      return __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
    } else if constexpr (P == 1) {
      return __builtin_amdgcn_mfma_f32_16x16x4f32((float)a[0], (float)b[0], c, 0, 0, 0);
    } else {
      v4s ah, bh, al, bl;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ah[u] = bf16_bits((float)a[u]);
        bh[u] = bf16_bits((float)b[u]);
        if constexpr (P == 2) {
          al[u] = bf16_bits((float)(a[u] - (double)bf16_float(ah[u])));
          bl[u] = bf16_bits((float)(b[u] - (double)bf16_float(bh[u])));
        }
      }
      c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, c, 0, 0, 0);
      if constexpr (P == 2) {
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, c, 0, 0, 0);
      }
      return c;
    }
  }
  static __device__ __forceinline__ int row(int v, int q) { return P ? 4 * q + v : 4 * v + q; }
};

// One 16 x 16 output tile accumulated over an inner dimension K: the
// operand fragments of U consecutive MFMA steps are loaded before those
// steps issue, so a wavefront keeps U loads of each operand in flight
// instead of one.  a_at(l) is op(A)(i, l) of this lane's row i, b_at(l) is
// op(B)(l, j) of its column j; lanes outside the tile (ia, jb false) and
// l >= K contribute zeros.
template <int P, class FA, class FB>
__device__ __forceinline__ void mfma_span(typename Mfma16<P>::acc_t& acc, int K, int q, bool ia, bool jb, FA a_at,
                                          FB b_at) {
  using M = Mfma16<P>;
  constexpr int U = P >= 2 ? 2 : 4;
  for (int l0 = 0; l0 < K; l0 += U * M::KG) {
    double a[U][M::EPL], b[U][M::EPL];
#pragma unroll
    for (int s = 0; s < U; ++s)
#pragma unroll
      for (int u = 0; u < M::EPL; ++u) {
        const int l = l0 + s * M::KG + M::kof(u, q);
        a[s][u] = (ia && l < K) ? a_at(l) : 0.0;
        b[s][u] = (jb && l < K) ? b_at(l) : 0.0;
      }
#pragma unroll
    for (int s = 0; s < U; ++s)
      if (l0 + s * M::KG < K) acc = M::step(a[s], b[s], acc);
  }
}

// One workgroup per output, or per run of kGemmTilesPerGroup tiles of a
// large output (work[2 g] = output, work[2 g + 1] = first tile; null work:
// workgroup g takes output g whole); the tiles are dealt to the four
// wavefronts (tile w, w + 4, ...), i fastest, and each tile sums all terms.
template <int P>
__global__ __launch_bounds__(256) void gemm_sum_kernel(const GemmOut* __restrict__ outs,
                                                       const GemmTerm* __restrict__ terms,
                                                       const int32_t* __restrict__ work) {
  using M = Mfma16<P>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int oi = work ? work[2 * blockIdx.x] : (int)blockIdx.x;
  const int tfirst = work ? work[2 * blockIdx.x + 1] : 0;
  const GemmOut o = outs[oi];
  if (o.m <= 0 || o.n <= 0 || (o.t0 == o.t1 && o.beta)) return;
  const int mt = (o.m + 15) / 16;
  const int tend = work ? min(mt * ((o.n + 15) / 16), tfirst + kGemmTilesPerGroup) : mt * ((o.n + 15) / 16);
  const int r = lane & 15, q = lane >> 4;
  for (int tile = tfirst + wave; tile < tend; tile += 4) {
    const int i0 = (tile % mt) * 16, j0 = (tile / mt) * 16;
    typename M::acc_t acc = M::zero();
    const int i = i0 + r, j = j0 + r;
    const bool ia = i < o.m, jb = j < o.n;
    for (int ti = o.t0; ti < o.t1; ++ti) {
      const GemmTerm T = terms[ti];
      double alpha = T.alpha;
      if (T.flags & GT_SCALE_MUL) {
        alpha *= *T.scale;
      } else if (T.flags & GT_SCALE_INV) {
        const double s = *T.scale;
        alpha = s > 0.0 ? alpha / s : 0.0;
      }
      const double* A = (const double*)T.A;
      const double* B = (const double*)T.B;
      const bool tA = T.flags & GT_TA, tB = T.flags & GT_TB;
      const int64_t sa_i = tA ? T.lda : 1, sa_l = tA ? 1 : T.lda;
      if (T.flags & GT_BEYE) {
        // op(A) times the identity: the tile's own entries of op(A), added in
        // the accumulator layout (no products, no re-reads across the tile)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ia_ = i0 + M::row(v, q), jc = j0 + r;
          if (ia_ < o.m && jc < o.n && jc < T.k) acc[v] += alpha * A[(int64_t)ia_ * sa_i + (int64_t)jc * sa_l];
        }
        continue;
      }
      const int64_t sb_l = tB ? T.ldb : 1, sb_j = tB ? 1 : T.ldb;
      const double* Ai = A + (int64_t)i * sa_i;
      const double* Bj = B + (int64_t)j * sb_j;
      mfma_span<P>(acc, T.k, q, ia, jb, [&](int l) { return Ai[(int64_t)l * sa_l] * alpha; },
                   [&](int l) { return Bj[(int64_t)l * sb_l]; });
    }
    double* C = (double*)o.C;
    const int jc = j0 + r;
    if (jc < o.n) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ic = i0 + M::row(v, q);
        if (ic < o.m) {
          double* p = C + ic + (int64_t)jc * o.ldc;
          *p = o.beta ? *p + (double)acc[v] : (double)acc[v];
        }
      }
    }
  }
}

void k_gemm_sum(const GemmOut* outs, const GemmTerm* terms, const int32_t* work, int ngroups, int prec,
                void* stream) {
  if (ngroups <= 0) return;
  auto k = prec == 1 ? gemm_sum_kernel<1> : prec == 2 ? gemm_sum_kernel<2> : prec == 3 ? gemm_sum_kernel<3>
                                                                                      : gemm_sum_kernel<0>;
  hipLaunchKernelGGL(k, dim3(ngroups), dim3(256), 0, (hipStream_t)stream, outs, terms, work);
  HIP_OK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// chained small products C = beta C + op(A) B op(D) (FP64 MFMA): one
// workgroup (4 wavefronts) per item; the 16 x 16 tiles of T = op(A) B are
// formed into LDS, then those of C from T and op(D)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void chain3_kernel(const Chain3* __restrict__ items) {
  __shared__ double Ts[kChain3Max * kChain3Max];  // T(i, l) at i + 64 l
  using M = Mfma16<0>;
  constexpr int KS = kChain3Max / 4;  // MFMA k-steps at most
  const Chain3 it = items[blockIdx.x];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, q4 = lane >> 4;
  const int mt = (it.m + 15) / 16, qt = (it.q + 15) / 16, nt = (it.n + 15) / 16;
  // each wavefront loads all operand fragments of a tile before its MFMA
  // steps, so the global loads of a tile overlap instead of forming a chain
  for (int tile = wave; tile < mt * qt; tile += 4) {
    const int i0 = (tile % mt) * 16, j0 = (tile / mt) * 16;
    const int i = i0 + r, j = j0 + r;
    double a[KS], b[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int l = 4 * ks + q4;
      a[ks] = 0.0;
      b[ks] = 0.0;
      if (l < it.p) {
        if (i < it.m) a[ks] = it.tA ? it.A[l + (int64_t)i * it.lda] : it.A[i + (int64_t)l * it.lda];
        if (j < it.q) b[ks] = it.B[l + (int64_t)j * it.ldb];
      }
    }
    typename M::acc_t acc = M::zero();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      if (4 * ks < it.p) acc = M::step(&a[ks], &b[ks], acc);
#pragma unroll
    for (int v = 0; v < 4; ++v) Ts[i0 + M::row(v, q4) + (j0 + r) * kChain3Max] = acc[v];
  }
  __syncthreads();
  for (int tile = wave; tile < mt * nt; tile += 4) {
    const int i0 = (tile % mt) * 16, j0 = (tile / mt) * 16;
    const int i = i0 + r, j = j0 + r;
    double a[KS], b[KS];
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int l = 4 * ks + q4;
      a[ks] = 0.0;
      b[ks] = 0.0;
      if (l < it.q) {
        if (i < it.m) a[ks] = Ts[i + l * kChain3Max];
        if (j < it.n) b[ks] = it.dT ? it.D[j + (int64_t)l * it.ldd] : it.D[l + (int64_t)j * it.ldd];
      }
    }
    typename M::acc_t acc = M::zero();
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
      if (4 * ks < it.q) acc = M::step(&a[ks], &b[ks], acc);
    if (j < it.n) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ic = i0 + M::row(v, q4);
        if (ic < it.m) {
          double* c = it.C + ic + (int64_t)j * it.ldc;
          *c = it.beta ? *c + acc[v] : acc[v];
        }
      }
    }
  }
}

void k_chain3(const Chain3* items, int n, void* stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(chain3_kernel, dim3(n), dim3(256), 0, (hipStream_t)stream, items);
  HIP_OK(hipGetLastError());
}

// Dynamic LDS of the factorization kernels.  Each kernel calls its body
// twice, once on a pointer into this array and once on global scratch, and
// the bodies are force-inlined: the compiler then sees the address space of
// every access and emits LDS instructions (ds_read / ds_write, counted
// separately from global loads) for the LDS copy.
extern __shared__ double lds_dyn[];

// ---------------------------------------------------------------------------
// grouped products over product-tree triples (MFMA): one wavefront per
// 16 x 16 output tile; each tile scans its block's triples and accumulates the
// ones of the launch's kind
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void gemm_tri_kernel(const TriOut* __restrict__ outs,
                                                       const int32_t* __restrict__ tiles, int ntiles,
                                                       const TriFamily F) {
  using M = Mfma16<P>;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tix = blockIdx.x * 4 + wave;
  if (tix >= ntiles) return;
  const int oi = tiles[3 * tix], i0 = tiles[3 * tix + 1], j0 = tiles[3 * tix + 2];
  const TriOut o = outs[oi];
  const int r = lane & 15, q = lane >> 4;
  typename M::acc_t acc = M::zero();
  const int i = i0 + r, j = j0 + r;
  const bool ia = i < o.m, jb = j < o.n;
  for (int t = o.q0; t < o.q1; ++t) {
    const int4 tr = reinterpret_cast<const int4*>(F.tri)[t];
    if (tr.w != F.kind) continue;
    const double* A = F.A[tr.y];
    const double* B = F.B[tr.z];
    const int64_t lda = F.lda[tr.y], ldb = F.ldb[tr.z];
    const int k = F.ks ? F.ks[tr.x] : F.k;
    const int64_t sa_i = F.tA ? lda : 1, sa_l = F.tA ? 1 : lda;
    const int64_t sb_l = F.tB ? ldb : 1, sb_j = F.tB ? 1 : ldb;
    const double* Ai = A + (int64_t)i * sa_i;
    const double* Bj = B + (int64_t)j * sb_j;
    mfma_span<P>(acc, k, q, ia, jb, [&](int l) { return Ai[(int64_t)l * sa_l]; },
                 [&](int l) { return Bj[(int64_t)l * sb_l]; });
  }
  double* C = o.C;
  const int jc = j0 + r;
  if (jc < o.n) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ic = i0 + M::row(v, q);
      if (ic < o.m) {
        double* p = C + ic + (int64_t)jc * o.ldc;
        *p = o.beta ? *p + (double)acc[v] : (double)acc[v];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Block form of the triple products for outputs up to 64 x 64 (the dense
// leaf blocks, or 64 x 64 parts of larger ones: rows ro.. of A times columns
// co.. of B): one workgroup per output, operands staged through LDS in
// k-chunks of 16 (A as loaded, B transposed so that both MFMA operands are
// read along consecutive lanes), each wavefront owning a 32 x 32 quadrant
// (2 x 2 tiles of 16 x 16).  Global loads run along columns (coalesced).
// ---------------------------------------------------------------------------
constexpr int kTriKC = 16;        // k-chunk
constexpr int kTriLdA = 64 + 1;   // LDS stride of the A chunk (odd: spreads banks)
constexpr int kTriLdB = kTriKC + 1;

template <int P>
__global__ __launch_bounds__(256) void gemm_tri_block_kernel(const TriOut* __restrict__ outs, const TriFamily F) {
  using M = Mfma16<P>;
  __shared__ double As[kTriKC * kTriLdA];  // A(i, l) at i + l * kTriLdA
  __shared__ double Bs[64 * kTriLdB];      // B(l, j) at l + j * kTriLdB
  const TriOut o = outs[blockIdx.x];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int r = lane & 15, q = lane >> 4;
  const int wi = (wave & 1) * 32, wj = (wave >> 1) * 32;  // quadrant of this wavefront
  typename M::acc_t acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = M::zero();
  // The output's (triple, chunk) sequence, software-pipelined: each thread
  // holds its share of the next chunk of A and B in registers, loaded while
  // the MFMA steps consume the current chunk from LDS.
  const int4* tri = reinterpret_cast<const int4*>(F.tri);
  auto next_triple = [&](int t) {  // first triple of this family at or after t (uniform)
    while (t < o.q1 && tri[t].w != F.kind) ++t;
    return t;
  };
  constexpr int kPer = 64 * kTriKC / 256;  // elements of each operand chunk per thread
  const double* A = nullptr;
  const double* B = nullptr;
  int64_t lda = 0, ldb = 0;
  int k = 0;
  auto bind = [&](int t) {
    const int4 tr = tri[t];
    lda = F.lda[tr.y];
    ldb = F.ldb[tr.z];
    A = F.A[tr.y] + o.ro;                 // rows ro.. of A
    B = F.B[tr.z] + (int64_t)o.co * ldb;  // columns co.. of B
    k = F.ks ? F.ks[tr.x] : F.k;
  };
  double ra[kPer], rb[kPer];
  // operands live in device memory: global loads (counted on vmcnt only)
  // stay in flight past the LDS reads of the MFMA steps, flat loads would not
  using gdouble = const __attribute__((address_space(1))) double;
  auto fetch = [&](int l0) {
    gdouble* Ag = (gdouble*)A;
    gdouble* Bg = (gdouble*)B;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      const int i = e & 63, la = e >> 6;                // A chunk: consecutive threads along i
      ra[u] = (i < o.m && l0 + la < k) ? Ag[i + (int64_t)(l0 + la) * lda] : 0.0;
      const int lb = e & (kTriKC - 1), j = e / kTriKC;  // B chunk: consecutive threads down a column
      rb[u] = (j < o.n && l0 + lb < k) ? Bg[(l0 + lb) + (int64_t)j * ldb] : 0.0;
    }
  };
  int t = next_triple(o.q0), l0 = 0;
  if (t < o.q1) {
    bind(t);
    fetch(0);
  }
  while (t < o.q1) {
    __syncthreads();  // previous chunk consumed
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + 256 * u;
      As[(e & 63) + (e >> 6) * kTriLdA] = ra[u];
      Bs[(e & (kTriKC - 1)) + (e / kTriKC) * kTriLdB] = rb[u];
    }
    __syncthreads();
    l0 += kTriKC;
    if (l0 >= k) {
      t = next_triple(t + 1);
      l0 = 0;
      if (t < o.q1) bind(t);
    }
    if (t < o.q1) fetch(l0);
#pragma unroll
    for (int ls = 0; ls < kTriKC; ls += M::KG) {
      double av[2][M::EPL], bv[2][M::EPL];
#pragma unroll
      for (int u = 0; u < M::EPL; ++u) {
        const int l = ls + M::kof(u, q);
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a][u] = As[(wi + 16 * a + r) + l * kTriLdA];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b][u] = Bs[l + (wj + 16 * b + r) * kTriLdB];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = M::step(av[a], bv[b], acc[a][b]);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int jc = wj + 16 * b + r;
      if (jc >= o.n) continue;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ic = wi + 16 * a + M::row(v, q);
        if (ic < o.m) {
          double* p = o.C + ic + (int64_t)jc * o.ldc;
          *p = o.beta ? *p + (double)acc[a][b][v] : (double)acc[a][b][v];
        }
      }
    }
}

void k_gemm_tri_block(const TriOut* outs, int nouts, const TriFamily& fam, int prec, void* stream) {
  if (nouts <= 0) return;
  H2_REQUIRE(!fam.tA && !fam.tB, H2_ERR_ARG, "gemm_tri_block: untransposed operands only");
  auto k = prec == 1   ? gemm_tri_block_kernel<1>
           : prec == 2 ? gemm_tri_block_kernel<2>
           : prec == 3 ? gemm_tri_block_kernel<3>
                       : gemm_tri_block_kernel<0>;
  hipLaunchKernelGGL(k, dim3(nouts), dim3(256), 0, (hipStream_t)stream, outs, fam);
  HIP_OK(hipGetLastError());
}

void k_gemm_tri(const TriOut* outs, const int32_t* tiles, int ntiles, const TriFamily& fam, int prec, void* stream) {
  if (ntiles <= 0) return;
  dim3 grid((ntiles + 3) / 4);
  auto k = prec == 1 ? gemm_tri_kernel<1> : prec == 2 ? gemm_tri_kernel<2> : prec == 3 ? gemm_tri_kernel<3>
                                                                                      : gemm_tri_kernel<0>;
  hipLaunchKernelGGL(k, grid, dim3(256), 0, (hipStream_t)stream, outs, tiles, ntiles, fam);
  HIP_OK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Fused formation of G's coefficients on one level of T^XY (see GformArgs):
// one workgroup per block, four wavefronts.  Each output of at most 64 x 64
// is cut into 16 x 16 tiles; wavefront w owns tiles w, w + 4, ... and keeps
// them in MFMA accumulators across all of the block's triples, reading the
// operand fragments from device memory (they are shared by many blocks and
// stay in L2).  TAA, TNA and the final Mm pass through LDS as operands of
// the closing products.
// ---------------------------------------------------------------------------
constexpr int kGformMaxTiles = 4;  // 16 tiles of a 64 x 64 output over 4 wavefronts

template <int P, class FA, class FB>
__device__ __forceinline__ void gform_tile(typename Mfma16<P>::acc_t& acc, int i0, int j0, int m, int n, int K,
                                           int r, int q, FA a_at, FB b_at) {
  const int i = i0 + r, j = j0 + r;
  mfma_span<P>(acc, K, q, i < m, j < n, [&](int l) { return a_at(i, l); }, [&](int l) { return b_at(l, j); });
}

template <int P, class FS>
__device__ __forceinline__ void gform_store(const typename Mfma16<P>::acc_t& acc, int i0, int j0, int m, int n, int r,
                                            int q, FS put) {
  using M = Mfma16<P>;
  const int j = j0 + r;
  if (j >= n) return;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = i0 + M::row(v, q);
    if (i < m) put(i, j, (double)acc[v]);
  }
}

template <int P>
__global__ __launch_bounds__(256) void gform_kernel(const GformArgs A) {
  using M = Mfma16<P>;
  using acc_t = typename M::acc_t;
  const int b = A.b0 + blockIdx.x;
  const int t = A.bt[2 * b] - A.c0, rr = A.bt[2 * b + 1] - A.c0;
  const int k = A.k, kt = A.krow[t], kr = A.kcol[rr];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  // LDS: TAA (k x k, ld k), TNA (ktmax x k, ld ktmax), Mm (k x krmax, ld k)
  double* Taa = lds_dyn;
  double* Tna = Taa + (size_t)k * k;
  double* Mm = Tna + (size_t)A.ktmax * k;
  const int tk = (k + 15) / 16, tkt = (kt + 15) / 16, tkr = (kr + 15) / 16;
  acc_t aa[kGformMaxTiles], na[kGformMaxTiles], an[kGformMaxTiles];
#pragma unroll
  for (int x = 0; x < kGformMaxTiles; ++x) aa[x] = na[x] = an[x] = M::zero();
  bool any_aa = false, any_na = false, any_an = false;
  const int4* tri = reinterpret_cast<const int4*>(A.tri);
  for (int p = A.tri_ptr[b]; p < A.tri_ptr[b + 1]; ++p) {
    const int4 T = tri[p];
    if (T.w == TK_AA) {  // S_X (P S_Y)
      any_aa = true;
      const double* X = A.SX[T.y];
      const int64_t lx = A.ldSX[T.y];
      const double* Y = A.PS[T.z];
#pragma unroll
      for (int x = 0; x < kGformMaxTiles; ++x) {
        const int tile = wave + 4 * x;
        if (tile >= tk * tk) break;
        gform_tile<P>(aa[x], (tile % tk) * 16, (tile / tk) * 16, k, k, k, r, q,
                      [&](int i, int l) { return X[i + (int64_t)l * lx]; },
                      [&](int l, int j) { return Y[l + (int64_t)j * k]; });
      }
    } else if (T.w == TK_NA && kt > 0) {  // A_{t,s} S_Y
      any_na = true;
      const double* X = A.Ar[T.y - A.bx0];
      const int64_t lx = A.ldAr[T.y - A.bx0];
      const double* Y = A.SY[T.z];
      const int64_t ly = A.ldSY[T.z];
#pragma unroll
      for (int x = 0; x < kGformMaxTiles; ++x) {
        const int tile = wave + 4 * x;
        if (tile >= tkt * tk) break;
        gform_tile<P>(na[x], (tile % tkt) * 16, (tile / tkt) * 16, kt, k, k, r, q,
                      [&](int i, int l) { return X[i + (int64_t)l * lx]; },
                      [&](int l, int j) { return Y[l + (int64_t)j * ly]; });
      }
    } else if (T.w == TK_AN && kr > 0) {  // S_X A^c^*
      any_an = true;
      const double* X = A.SX[T.y];
      const int64_t lx = A.ldSX[T.y];
      const double* Y = A.Ac[T.z - A.by0];
      const int64_t ly = A.ldAc[T.z - A.by0];
#pragma unroll
      for (int x = 0; x < kGformMaxTiles; ++x) {
        const int tile = wave + 4 * x;
        if (tile >= tk * tkr) break;
        gform_tile<P>(an[x], (tile % tk) * 16, (tile / tk) * 16, k, kr, k, r, q,
                      [&](int i, int l) { return X[i + (int64_t)l * lx]; },
                      [&](int l, int j) { return Y[j + (int64_t)l * ly]; });
      }
    }
  }
  // TAA and TNA to LDS (zero where the block has no such triple)
#pragma unroll
  for (int x = 0; x < kGformMaxTiles; ++x) {
    const int tile = wave + 4 * x;
    if (tile < tk * tk)
      gform_store<P>(aa[x], (tile % tk) * 16, (tile / tk) * 16, k, k, r, q,
                     [&](int i, int j, double v) { Taa[i + j * k] = any_aa ? v : 0.0; });
    if (tile < tkt * tk)
      gform_store<P>(na[x], (tile % tkt) * 16, (tile / tkt) * 16, kt, k, r, q,
                     [&](int i, int j, double v) { Tna[i + j * A.ktmax] = any_na ? v : 0.0; });
  }
  __syncthreads();
  const double* Rc = A.Rc[rr];
  const int64_t lrc = kr > 1 ? kr : 1;
  // Mm = TAA R^c^* + MAN (k x kr), to LDS
#pragma unroll
  for (int x = 0; x < kGformMaxTiles; ++x) {
    const int tile = wave + 4 * x;
    if (tile >= tk * tkr) break;
    acc_t m = any_an ? an[x] : M::zero();
    if (any_aa)
      gform_tile<P>(m, (tile % tk) * 16, (tile / tk) * 16, k, kr, k, r, q,
                    [&](int i, int l) { return Taa[i + l * k]; },
                    [&](int l, int j) { return Rc[j + (int64_t)l * lrc]; });
    gform_store<P>(m, (tile % tk) * 16, (tile / tk) * 16, k, kr, r, q,
                   [&](int i, int j, double v) { Mm[i + j * k] = v; });
  }
  __syncthreads();
  // S = TNA R^c^* + R_t Mm (kt x kr), to device memory
  if (kt == 0 || kr == 0) return;
  const double* Rt = A.Rr[t];
  const int64_t lrt = kt > 1 ? kt : 1;
  double* S = A.S[blockIdx.x];
  const int ntile = tkt * tkr;
  for (int tile = wave; tile < ntile; tile += 4) {
    acc_t s = M::zero();
    const int i0 = (tile % tkt) * 16, j0 = (tile / tkt) * 16;
    if (any_na)
      gform_tile<P>(s, i0, j0, kt, kr, k, r, q, [&](int i, int l) { return Tna[i + l * A.ktmax]; },
                    [&](int l, int j) { return Rc[j + (int64_t)l * lrc]; });
    if (any_aa || any_an)
      gform_tile<P>(s, i0, j0, kt, kr, k, r, q, [&](int i, int l) { return Rt[i + (int64_t)l * lrt]; },
                    [&](int l, int j) { return Mm[l + j * k]; });
    gform_store<P>(s, i0, j0, kt, kr, r, q, [&](int i, int j, double v) { S[i + (int64_t)j * lrt] = v; });
  }
}

size_t gform_lds_doubles(int k, int ktmax, int krmax) {
  return (size_t)k * k + (size_t)ktmax * k + (size_t)k * krmax;
}

void k_gform(const GformArgs& a, int nblocks, int prec, void* stream) {
  if (nblocks <= 0) return;
  H2_REQUIRE(a.k <= 64 && a.ktmax <= 64 && a.krmax <= 64, H2_ERR_ARG, "gform: dimensions above 64");
  const size_t lds = gform_lds_doubles(a.k, std::max(a.ktmax, 1), std::max(a.krmax, 1)) * sizeof(double);
  H2_REQUIRE(lds <= (size_t)lds_limit_doubles() * sizeof(double), H2_ERR_ARG, "gform: LDS above the device's limit");
  auto kern = prec == 1 ? gform_kernel<1> : prec == 2 ? gform_kernel<2> : prec == 3 ? gform_kernel<3> : gform_kernel<0>;
  hipLaunchKernelGGL(kern, dim3(nblocks), dim3(256), lds, (hipStream_t)stream, a);
  HIP_OK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Householder QR of one m x n matrix W (ld) by a 256-thread workgroup
// ---------------------------------------------------------------------------
__device__ __forceinline__ void householder_qr(double* W, int64_t ld, int m, int n, double* tau, double* red) {
  const int tid = threadIdx.x;
  const int kmax = m < n ? m : n;
  for (int jj = 0; jj < kmax; ++jj) {
    double s = 0.0;
    for (int i = jj + 1 + tid; i < m; i += 256) {
      const double x = W[i + jj * ld];
      s += x * x;
    }
    s = block_sum(s, red);
    const double alpha = W[jj + jj * ld];
    double t, beta, scal;
    if (s == 0.0) {
      t = 0.0;
      beta = alpha;
      scal = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + s), alpha);
      t = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    __syncthreads();
    for (int i = jj + 1 + tid; i < m; i += 256) W[i + jj * ld] *= scal;
    if (tid == 0) {
      W[jj + jj * ld] = beta;
      if (tau) tau[jj] = t;
    }
    __syncthreads();
    if (t != 0.0) {
      // trailing update: each of the nt columns is owned by a group of tpc
      // lanes (a power of two dividing 64) that splits its rows and reduces
      // with log2(tpc) shuffles
      const int nt = n - jj - 1;
      int tpc = 64;
      while (tpc > 1 && tpc * nt > 256) tpc >>= 1;
      const int grp = tid / tpc, gl = tid % tpc, ngrp = 256 / tpc;
      const double* v = W + jj * ld;
      for (int c0 = 0; c0 < nt; c0 += ngrp) {
        const int c = jj + 1 + c0 + grp;
        const bool live = c0 + grp < nt;
        double d0 = 0.0, d1 = 0.0;
        double* wc = W + (int64_t)c * ld;
        if (live) {
          if (gl == 0) d0 = wc[jj];
          int i = jj + 1 + gl;
          for (; i + tpc < m; i += 2 * tpc) {
            d0 += v[i] * wc[i];
            d1 += v[i + tpc] * wc[i + tpc];
          }
          if (i < m) d0 += v[i] * wc[i];
        }
        const double d_ = group_sum(d0 + d1, tpc);
        if (live) {
          const double d = d_ * t;
          if (gl == 0) wc[jj] -= d;
#pragma unroll 4
          for (int i = jj + 1 + gl; i < m; i += tpc) wc[i] -= d * v[i];
        }
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// LDS capacity
// ---------------------------------------------------------------------------
__global__ void qr_kernel(const QrProb* __restrict__ probs, int lds_cap);
__global__ void apply_kernel(const ApplyProb* __restrict__ probs, const int32_t* __restrict__ work, int lds_cap);
__global__ void tsqr_kernel(const TsqrProb* __restrict__ probs, int nprob, double* __restrict__ scratch,
                            size_t slot, int lds_cap);
template <int NT>
__global__ void jacobi_kernel(const JacobiProb* __restrict__ probs, int nprob, double* __restrict__ scratch,
                              size_t slot, int lds_cap);
__global__ void jacobi_small_kernel(const JacobiProb* __restrict__ probs, int nprob, int per);
__global__ void norm2_kernel(const Norm2Prob* __restrict__ probs, int nprob, int per, int cshift);
template <int G, int CPT, int RPT>
__global__ void tsqr_rb_kernel(const TsqrProb* __restrict__ probs, int nprob);

int lds_limit_doubles() {
  // computed once (thread-safe static initialisation): the passes run on two
  // host threads
  static const int limit = [] {
    int dev = 0, maxb = 0;
    HIP_OK(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&maxb, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) maxb = 65536;
    // 2 KiB stay for static shared data
    int bytes = std::max(std::min(maxb, 160 * 1024) - 2048, 32 * 1024);
    const void* ks[] = {(const void*)qr_kernel, (const void*)apply_kernel, (const void*)tsqr_kernel,
                        (const void*)jacobi_kernel<256>, (const void*)jacobi_kernel<1024>,
                        (const void*)jacobi_small_kernel, (const void*)norm2_kernel,
                        (const void*)tsqr_rb_kernel<16, 1, 8>, (const void*)tsqr_rb_kernel<8, 1, 16>,
                        (const void*)tsqr_rb_kernel<8, 2, 8>, (const void*)gform_kernel<0>,
                        (const void*)gform_kernel<1>, (const void*)gform_kernel<2>, (const void*)gform_kernel<3>};
    for (const void* k : ks)
      if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) {
        (void)hipGetLastError();
        bytes = std::min(bytes, 64 * 1024 - 2048);
      }
    return bytes / 8;
  }();
  return limit;
}

// ---------------------------------------------------------------------------
// QR with reflectors
// ---------------------------------------------------------------------------
size_t qr_need_doubles(int m, int n) { return (size_t)m * n; }

__device__ __forceinline__ void qr_copy_r(const QrProb& P, const double* W, int64_t ld) {
  for (int64_t e = threadIdx.x; e < (int64_t)P.rrows * P.n; e += 256) {
    const int i = (int)(e % P.rrows), c = (int)(e / P.rrows);
    P.R[i + c * P.ldr] = (i <= c && i < P.m) ? W[i + c * ld] : 0.0;
  }
}

__global__ __launch_bounds__(256) void qr_kernel(const QrProb* __restrict__ probs, int lds_cap) {
  __shared__ double red[4];
  const QrProb P = probs[blockIdx.x];
  const int m = P.m, n = P.n, tid = threadIdx.x;
  if ((int64_t)m * n <= lds_cap) {
    double* W = lds_dyn;
    for (int64_t e = tid; e < (int64_t)m * n; e += 256) W[e] = P.A[(e % m) + (e / m) * P.lda];
    __syncthreads();
    householder_qr(W, m, m, n, P.tau, red);
    for (int64_t e = tid; e < (int64_t)m * n; e += 256) P.A[(e % m) + (e / m) * P.lda] = W[e];
    if (P.R) qr_copy_r(P, W, m);
  } else {
    householder_qr(P.A, P.lda, m, n, P.tau, red);
    if (P.R) qr_copy_r(P, P.A, P.lda);
  }
}

void k_qr(const QrProb* probs, int n, int lds_doubles, void* stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(qr_kernel, dim3(n), dim3(256), (size_t)lds_doubles * 8, (hipStream_t)stream, probs,
                     lds_doubles);
  HIP_OK(hipGetLastError());
}

// C <- Q^T C or Q C for the columns c0 .. c0+63, one wave per column
__device__ __forceinline__ void apply_cols(const ApplyProb& P, const double* V, int64_t ldv, const double* tau_s,
                                           int c0) {
  const int m = P.m, r = P.nrefl, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cend = min(P.ncols, c0 + 64);
  for (int c = c0 + wave; c < cend; c += 4) {
    double* C = P.C + (int64_t)c * P.ldc;
    for (int s = 0; s < r; ++s) {
      const int jj = P.trans ? s : r - 1 - s;
      const double t = tau_s[jj];
      if (t == 0.0) continue;
      const double* v = V + jj * ldv;
      double d = 0.0;
#pragma unroll 2
      for (int i = jj + lane; i < m; i += 64) d += (i == jj ? 1.0 : v[i]) * C[i];
      d = wave_sum(d) * t;
#pragma unroll 2
      for (int i = jj + lane; i < m; i += 64) C[i] -= d * (i == jj ? 1.0 : v[i]);
    }
  }
}

// The same with each column held in registers (EPL = ceil(m / 64) elements
// per lane) across all reflectors: one read and one write of C per column.
template <int EPL>
__device__ __forceinline__ void apply_cols_reg(const ApplyProb& P, const double* V, int64_t ldv,
                                               const double* tau_s, int c0) {
  const int m = P.m, r = P.nrefl, wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cend = min(P.ncols, c0 + 64);
  for (int c = c0 + wave; c < cend; c += 4) {
    double* C = P.C + (int64_t)c * P.ldc;
    double x[EPL];
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int i = lane + 64 * e;
      x[e] = i < m ? C[i] : 0.0;
    }
    for (int s = 0; s < r; ++s) {
      const int jj = P.trans ? s : r - 1 - s;
      const double t = tau_s[jj];
      if (t == 0.0) continue;
      const double* v = V + jj * ldv;
      double ve[EPL];
      double d = 0.0;
#pragma unroll
      for (int e = 0; e < EPL; ++e) {
        const int i = lane + 64 * e;
        ve[e] = (i < jj || i >= m) ? 0.0 : (i == jj ? 1.0 : v[i]);
        d += ve[e] * x[e];
      }
      d = wave_sum(d) * t;
#pragma unroll
      for (int e = 0; e < EPL; ++e) x[e] -= d * ve[e];
    }
#pragma unroll
    for (int e = 0; e < EPL; ++e) {
      const int i = lane + 64 * e;
      if (i < m) C[i] = x[e];
    }
  }
}

template <int EPL>
__device__ __forceinline__ void apply_dispatch(const ApplyProb& P, const double* V, int64_t ldv,
                                               const double* tau_s, int c0) {
  if constexpr (EPL == 0)
    apply_cols(P, V, ldv, tau_s, c0);
  else
    apply_cols_reg<EPL>(P, V, ldv, tau_s, c0);
}

template <int EPL>
__device__ __forceinline__ void apply_body(const ApplyProb& P, int c0, int lds_cap, const double* tau_s) {
  const int m = P.m, r = P.nrefl;
  if ((int64_t)m * r <= lds_cap) {
    for (int64_t e = threadIdx.x; e < (int64_t)m * r; e += 256) lds_dyn[e] = P.V[(e % m) + (e / m) * P.ldv];
    __syncthreads();
    apply_dispatch<EPL>(P, lds_dyn, m, tau_s, c0);
  } else {
    __syncthreads();
    apply_dispatch<EPL>(P, P.V, P.ldv, tau_s, c0);
  }
}

// work item = (problem, first column); 64 columns per item
__global__ __launch_bounds__(256) void apply_kernel(const ApplyProb* __restrict__ probs,
                                                    const int32_t* __restrict__ work, int lds_cap) {
  __shared__ double tau_s[256];
  const ApplyProb P = probs[work[2 * blockIdx.x]];
  const int c0 = work[2 * blockIdx.x + 1];
  const int m = P.m, r = P.nrefl, tid = threadIdx.x;
  for (int e = tid; e < r; e += 256) tau_s[e] = P.tau[e];
  if (m <= 64)
    apply_body<1>(P, c0, lds_cap, tau_s);
  else if (m <= 128)
    apply_body<2>(P, c0, lds_cap, tau_s);
  else if (m <= 256)
    apply_body<4>(P, c0, lds_cap, tau_s);
  else if (m <= 512)
    apply_body<8>(P, c0, lds_cap, tau_s);
  else
    apply_body<0>(P, c0, lds_cap, tau_s);
}

void k_apply(const ApplyProb* probs, const int32_t* work, int nwork, int lds_doubles, void* stream) {
  if (nwork <= 0) return;
  hipLaunchKernelGGL(apply_kernel, dim3(nwork), dim3(256), (size_t)lds_doubles * 8, (hipStream_t)stream,
                     probs, work, lds_doubles);
  HIP_OK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// TSQR: R factor of T (N x me), T streamed in chunks of ch rows.  The running
// R (me x me, upper triangular, zero rows where no data has arrived yet) sits
// on top of the chunk; column jj of [R; C] is reduced by one Householder
// reflector whose vector is e_jj on the R part and C(:, jj) / (alpha - beta)
// on the chunk part, so each step touches row jj of R and the chunk only.
// ---------------------------------------------------------------------------
constexpr int kTsqrThreads = 512;        // register-blocked variants
constexpr int kTsqrStreamThreads = 1024;  // streaming kernel: one problem per 1024-thread workgroup
constexpr int kTsqrScratchChunk = 64;

// chunk rows of an m-column problem held in LDS of `cap` doubles together
// with its R factor; 0: no fit
static __host__ __device__ inline int tsqr_lds_chunk(int m, int cap) {
  const int mm = m > 0 ? m : 1;
  int c = cap / mm - mm;
  if (c > 256) c = 256;
  c &= ~31;
  return c >= 32 ? c : 0;
}
// chunk rows of a problem whose R factor does not fit beside them: the
// chunks alone in LDS (R in the global scratch slot), as many rows as fit,
// up to 128 in steps of 16; 0: no fit
static __host__ __device__ inline int tsqr_chunk_rows(int m, int cap) {
  const int mm = m > 0 ? m : 1;
  int c = cap / mm;
  if (c > 128) c = 128;
  c &= ~15;
  return c >= 32 ? c : 0;
}

size_t tsqr_lds_need(int m, int cap) {
  const int c = tsqr_lds_chunk(m, cap);
  return c ? (size_t)(m + c) * m : 0;
}
size_t tsqr_scratch_need(int m) { return (size_t)(m + kTsqrScratchChunk) * m; }
size_t tsqr_chunk_need(int m, int cap) { return (size_t)tsqr_chunk_rows(m, cap) * m; }

__device__ __forceinline__ double tsqr_src(const TsqrProb& P, int64_t idx) {
  return P.prec ? (double)((const float*)P.A)[idx] : ((const double*)P.A)[idx];
}

// one problem with N > me: R (me x me, leading dimension ldr) in Rw and the
// row chunks (at most ch x me, leading dimension ldc) in C; each lies in LDS
// or in the workgroup's global scratch slot
__device__ __forceinline__ void tsqr_reduce(const TsqrProb& P, double* Rw, int64_t ldr, double* C, int64_t ldc,
                                            int ch, int me, int off, double* red) {
  const int tid = threadIdx.x, wave = tid >> 6;
  const int m = P.m, N = P.N;
  for (int e = tid; e < me * me; e += kTsqrStreamThreads) Rw[(e % me) + (int64_t)(e / me) * ldr] = 0.0;
  for (int q0 = 0; q0 < N; q0 += ch) {
    const int cr = min(ch, N - q0);
    if (P.transA) {  // T(i, j) = A[j + i lda], consecutive threads along j
      for (int e = tid; e < cr * me; e += kTsqrStreamThreads) {
        const int j = e % me, i = e / me;
        C[i + (int64_t)j * ldc] = tsqr_src(P, off + j + (int64_t)(q0 + i) * P.lda);
      }
    } else {
      for (int e = tid; e < cr * me; e += kTsqrStreamThreads) {
        const int i = e % cr, j = e / cr;
        C[i + (int64_t)j * ldc] = tsqr_src(P, (q0 + i) + (int64_t)(off + j) * P.lda);
      }
    }
    __syncthreads();
    for (int jj = 0; jj < me; ++jj) {
      const double* cj = C + (int64_t)jj * ldc;
      double s = 0.0;
      for (int i = tid; i < cr; i += kTsqrStreamThreads) s += cj[i] * cj[i];
      s = wave_sum(s);
      if ((tid & 63) == 0) red[wave] = s;
      __syncthreads();
      s = 0.0;
#pragma unroll
      for (int w = 0; w < kTsqrStreamThreads / 64; ++w) s += red[w];
      const double alpha = Rw[jj + (int64_t)jj * ldr];
      if (s > 0.0) {
        const double beta = -copysign(sqrt(alpha * alpha + s), alpha);
        const double tau = (beta - alpha) / beta;
        const double scal = 1.0 / (alpha - beta);  // v = [1; scal * C(:, jj)]
        const int nt = me - jj - 1;
        int tpc = 64;
        while (tpc > 1 && tpc * nt > kTsqrStreamThreads) tpc >>= 1;
        const int grp = tid / tpc, gl = tid % tpc, ngrp = kTsqrStreamThreads / tpc;
        for (int c0 = 0; c0 < nt; c0 += ngrp) {
          const int c = jj + 1 + c0 + grp;
          const bool live = c0 + grp < nt;
          double d0 = 0.0, d1 = 0.0;
          double* cc = C + (int64_t)c * ldc;
          if (live) {
            int i = gl;
            for (; i + tpc < cr; i += 2 * tpc) {
              d0 += cj[i] * cc[i];
              d1 += cj[i + tpc] * cc[i + tpc];
            }
            if (i < cr) d0 += cj[i] * cc[i];
          }
          const double dsum = group_sum(d0 + d1, tpc);
          if (live) {
            double* rj = Rw + jj + (int64_t)c * ldr;
            const double d = tau * (*rj + scal * dsum);
            if (gl == 0) *rj -= d;
            const double f = d * scal;
#pragma unroll 4
            for (int i = gl; i < cr; i += tpc) cc[i] -= f * cj[i];
          }
        }
        if (tid == 0) Rw[jj + (int64_t)jj * ldr] = beta;
      }
      __syncthreads();
    }
  }
  const int p = min(N, m);
  for (int e = tid; e < p * m; e += kTsqrStreamThreads) {
    const int i = e % p, j = e / p;
    P.R[i + (int64_t)j * P.ldr] = (i <= j && j < me) ? Rw[i + (int64_t)j * ldr] : 0.0;
  }
}

__global__ __launch_bounds__(kTsqrStreamThreads) void tsqr_kernel(const TsqrProb* __restrict__ probs, int nprob,
                                                            double* __restrict__ scratch, size_t slot,
                                                            int lds_cap) {
  __shared__ double red[kTsqrStreamThreads / 64];
  const int tid = threadIdx.x;
  for (int pi = blockIdx.x; pi < nprob; pi += gridDim.x) {
    const TsqrProb P = probs[pi];
    const int m = P.m, N = P.N;
    const int off = P.col_off ? min(max(*P.col_off, 0), m) : 0;
    const int me = m - off;
    const int p = min(N, m);
    if (N <= me) {
      // T itself is a factor with T^T T = R^T R (N rows): no reduction.  (The
      // structured step needs N > me: with fewer rows its R is not confined
      // to the first N rows.)
      for (int e = tid; e < p * m; e += kTsqrStreamThreads) {
        const int i = e % p, j = e / p;
        double v = 0.0;
        if (j < me) v = tsqr_src(P, P.transA ? off + j + (int64_t)i * P.lda : i + (int64_t)(off + j) * P.lda);
        P.R[i + (int64_t)j * P.ldr] = v;
      }
      if (tid == 0 && P.work) *P.work = 0.0;
    } else {
      const int ch = tsqr_lds_chunk(m, lds_cap), chh = tsqr_chunk_rows(m, lds_cap);
      double* slot_p = scratch + (size_t)blockIdx.x * slot;
      if (ch > 0)  // R and the chunks in LDS
        tsqr_reduce(P, lds_dyn, me + ch, lds_dyn + me, me + ch, ch, me, off, red);
      else if (chh > 0)  // R in the global scratch slot, the chunks in LDS
        tsqr_reduce(P, slot_p, me, lds_dyn, chh, chh, me, off, red);
      else
        tsqr_reduce(P, slot_p, me + kTsqrScratchChunk, slot_p + me, me + kTsqrScratchChunk, kTsqrScratchChunk, me,
                    off, red);
      if (tid == 0 && P.work) {  // Householder QR of an N x me matrix
        const double dn = N, dm = me;
        *P.work = 2.0 * dn * dm * dm - 2.0 * dm * dm * dm / 3.0;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Register-blocked TSQR for m - off <= 128 (one problem per 512-thread
// workgroup).  Each column of the chunk belongs to a slot of G adjacent lanes
// that hold its rows in registers (RPT each); a slot holds CPT columns.  Per
// column jj the owning slot forms the reflector, one barrier publishes it
// (double-buffered), and every slot updates its own columns in registers.
// The chunk is loaded from global memory straight into the registers (the G
// lanes of a slot read G consecutive rows of a column, or of a row for the
// transposed input); LDS holds only R (me x me) and two reflector buffers,
// so several workgroups share a compute unit.
// ---------------------------------------------------------------------------
template <int G, int CPT, int RPT>
struct TsqrRB {
  static constexpr int kSlots = kTsqrThreads / G;
  static constexpr int kCH = G * RPT;
  static __host__ __device__ size_t need(int me) { return (size_t)(me + 1) * me + 2 * kCH + 4; }
};
using TsqrRB16 = TsqrRB<16, 1, 8>;  // me <= 32
using TsqrRB64 = TsqrRB<8, 1, 16>;  // me <= 64
using TsqrRB128 = TsqrRB<8, 2, 8>;  // me <= 128

// Lane rg of a slot holds the chunk rows rg, rg + G, rg + 2G, ...: the G lanes
// reading one reflector entry each then hit G consecutive doubles (distinct
// LDS banks).  R is stored with the odd leading dimension me + 1 so that the
// slots of a wavefront reading row jj of R hit distinct banks as well.
template <int G, int CPT, int RPT>
__global__ __launch_bounds__(kTsqrThreads) void tsqr_rb_kernel(const TsqrProb* __restrict__ probs, int nprob) {
  using K = TsqrRB<G, CPT, RPT>;
  constexpr int CH = K::kCH, SL = K::kSlots;
  const int tid = threadIdx.x;
  const int slot = tid / G, rg = tid % G;
  for (int pi = blockIdx.x; pi < nprob; pi += gridDim.x) {
    const TsqrProb P = probs[pi];
    const int m = P.m, N = P.N;
    const int off = P.col_off ? min(max(*P.col_off, 0), m) : 0;
    const int me = m - off;
    const int p = min(N, m);
    if (N <= me) {  // T itself is a factor (see tsqr_kernel)
      for (int e = tid; e < p * m; e += kTsqrThreads) {
        const int i = e % p, j = e / p;
        double v = 0.0;
        if (j < me) v = tsqr_src(P, P.transA ? off + j + (int64_t)i * P.lda : i + (int64_t)(off + j) * P.lda);
        P.R[i + (int64_t)j * P.ldr] = v;
      }
      if (tid == 0 && P.work) *P.work = 0.0;
      __syncthreads();
      continue;
    }
    const int ldr = me + 1;
    double* R = lds_dyn;          // me x me, column-major, ld me + 1
    double* vb = R + ldr * me;    // 2 x CH reflector buffers (by chunk row)
    double* sc = vb + 2 * CH;     // tau per buffer
    for (int e = tid; e < ldr * me; e += kTsqrThreads) R[e] = 0.0;
    __syncthreads();
    for (int q0 = 0; q0 < N; q0 += CH) {
      const int cr = min(CH, N - q0);
      // rows rg + G k of the slot's columns (T(i, j) = A[j + i lda] when transposed)
      double C[CPT][RPT];
#pragma unroll
      for (int cc = 0; cc < CPT; ++cc) {
        const int col = slot + SL * cc;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
          const int i = rg + G * k;
          double x = 0.0;
          if (col < me && i < cr)
            x = tsqr_src(P, P.transA ? off + col + (int64_t)(q0 + i) * P.lda : (q0 + i) + (int64_t)(off + col) * P.lda);
          C[cc][k] = x;
        }
      }
      for (int jj = 0; jj < me; ++jj) {
        const int buf = jj & 1;
        const int os = jj % SL, oc = jj / SL;
        // row jj of R for this slot's columns: final before step jj (prefetch)
        double rv[CPT];
#pragma unroll
        for (int cc = 0; cc < CPT; ++cc) {
          const int col = slot + SL * cc;
          rv[cc] = (col > jj && col < me) ? R[jj + col * ldr] : 0.0;
        }
        if (slot == os) {
          double s0 = 0.0, s1 = 0.0;
#pragma unroll
          for (int k = 0; k < RPT; k += 2) {
            const double x0 = (CPT == 1 || oc == 0) ? C[0][k] : C[CPT - 1][k];
            s0 += x0 * x0;
            if (k + 1 < RPT) {
              const double x1 = (CPT == 1 || oc == 0) ? C[0][k + 1] : C[CPT - 1][k + 1];
              s1 += x1 * x1;
            }
          }
          const double s = group_sum(s0 + s1, G);
          const double alpha = R[jj + jj * ldr];
          double tau = 0.0, scal = 0.0;
          if (s > 0.0) {
            const double beta = -copysign(sqrt(alpha * alpha + s), alpha);
            tau = (beta - alpha) / beta;
            scal = 1.0 / (alpha - beta);
            if (rg == 0) R[jj + jj * ldr] = beta;
          }
#pragma unroll
          for (int k = 0; k < RPT; ++k) {
            const double x = (CPT == 1 || oc == 0) ? C[0][k] : C[CPT - 1][k];
            vb[buf * CH + rg + G * k] = x * scal;
          }
          if (rg == 0) sc[buf] = tau;
        }
        __syncthreads();
        const double tau = sc[buf];
        double v[RPT];
#pragma unroll
        for (int k = 0; k < RPT; ++k) v[k] = vb[buf * CH + rg + G * k];
        if (tau != 0.0) {
#pragma unroll
          for (int cc = 0; cc < CPT; ++cc) {
            const int col = slot + SL * cc;
            if (col > jj && col < me) {  // uniform within the slot's G lanes
              double d0 = 0.0, d1 = 0.0;
#pragma unroll
              for (int k = 0; k < RPT; k += 2) {
                d0 += v[k] * C[cc][k];
                if (k + 1 < RPT) d1 += v[k + 1] * C[cc][k + 1];
              }
              const double d = group_sum(d0 + d1, G);
              const double dd = tau * (rv[cc] + d);
              if (rg == 0) R[jj + col * ldr] = rv[cc] - dd;
#pragma unroll
              for (int k = 0; k < RPT; ++k) C[cc][k] -= dd * v[k];
            }
          }
        }
      }
      __syncthreads();
    }
    for (int e = tid; e < p * m; e += kTsqrThreads) {
      const int i = e % p, j = e / p;
      P.R[i + (int64_t)j * P.ldr] = (i <= j && j < me) ? R[i + j * ldr] : 0.0;
    }
    if (tid == 0 && P.work) {  // Householder QR of an N x me matrix
      const double dn = N, dm = me;
      *P.work = 2.0 * dn * dm * dm - 2.0 * dm * dm * dm / 3.0;
    }
    __syncthreads();
  }
}

int tsqr_rb_variant(int m, int cap) {
  if (m <= 32 && TsqrRB16::need(m) <= (size_t)cap) return 1;
  if (m <= 64 && TsqrRB64::need(m) <= (size_t)cap) return 2;
  if (m <= 128 && TsqrRB128::need(m) <= (size_t)cap) return 3;
  return 0;
}

int tsqr_rb_chunk(int variant) {
  switch (variant) {
    case 1: return TsqrRB16::kCH;
    case 2: return TsqrRB64::kCH;
    case 3: return TsqrRB128::kCH;
  }
  return 0;
}

size_t tsqr_rb_need(int variant, int m) {
  switch (variant) {
    case 1: return TsqrRB16::need(m);
    case 2: return TsqrRB64::need(m);
    case 3: return TsqrRB128::need(m);
  }
  return 0;
}

void k_tsqr_rb(int variant, const TsqrProb* probs, int n, size_t lds_doubles, void* stream) {
  if (n <= 0) return;
  H2_REQUIRE(lds_doubles <= (size_t)lds_limit_doubles(), H2_ERR_ARG, "tsqr: LDS request over the limit");
  const size_t bytes = lds_doubles * 8;
  switch (variant) {
    case 1:
      hipLaunchKernelGGL((tsqr_rb_kernel<16, 1, 8>), dim3(n), dim3(kTsqrThreads), bytes, (hipStream_t)stream, probs, n);
      break;
    case 2:
      hipLaunchKernelGGL((tsqr_rb_kernel<8, 1, 16>), dim3(n), dim3(kTsqrThreads), bytes, (hipStream_t)stream, probs, n);
      break;
    case 3:
      hipLaunchKernelGGL((tsqr_rb_kernel<8, 2, 8>), dim3(n), dim3(kTsqrThreads), bytes, (hipStream_t)stream, probs, n);
      break;
    default:
      fail(H2_ERR_ARG, "tsqr: unknown variant");
  }
  HIP_OK(hipGetLastError());
}

void k_tsqr(const TsqrProb* probs, int n, size_t lds_doubles, size_t slot, double* scratch, void* stream) {
  if (n <= 0) return;
  H2_REQUIRE(slot == 0 || scratch, H2_ERR_ARG, "tsqr: global scratch missing");
  const int grid = slot == 0 ? n : std::min(n, 1024);
  hipLaunchKernelGGL(tsqr_kernel, dim3(grid), dim3(kTsqrStreamThreads), lds_doubles * 8, (hipStream_t)stream, probs,
                     n, scratch, slot, lds_limit_doubles());
  HIP_OK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// one-sided (Hestenes) Jacobi SVD of R, round-robin parallel ordering.
//  mode 0: rotate the columns s0..m-1 of R (p x m; columns < s0 are zero) and
//          accumulate the rotations: U = right singular vectors, all m of them
//  mode 1: rotate the rows of R' (pe x me, pe = min(p, me), me = m - s0), i.e.
//          the columns of R'^T; at convergence column j of R'^T V equals
//          sigma_j v_j with v_j a right singular vector of R', so U needs no
//          accumulation.  Triangular factors converge in far fewer sweeps
//          this way.  U(:, pos) = [0 (s0 rows); v_j] for pos < pe, else 0.
// Singular values = column norms, sorted descending (ties by index).
// ---------------------------------------------------------------------------
static __host__ __device__ inline int pow2ceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}
// lanes per pair for nt threads (at least gmin): all pairs of a round at
// once where possible
static __host__ __device__ inline int jacobi_gsz(int npairs, int nt, int gmin) {
  int g = 64;
  while (g > gmin && g * npairs > nt) g >>= 1;
  return g;
}
// Column stride of the rotated matrix.  Rows len .. L-1 (L = max(gsz,
// pow2ceil(len))) are kept zero, so each lane's EPL = L / gsz elements are
// loaded without per-element predicates.  The extra shift by gsz (for gsz <
// 32) makes the lane groups of a wavefront, which read consecutive columns,
// fall on different LDS banks.
static __host__ __device__ inline int jacobi_ld(int len, int gsz) {
  const int L = max(gsz, pow2ceil(len));
  return L + (gsz < 32 ? gsz : 0);
}
static __host__ __device__ inline size_t jacobi_ld_max(int len) {
  return (size_t)max(64, pow2ceil(len)) + 16;
}
static __host__ __device__ inline size_t jacobi_need(int p, int m, int mode) {
  // mode 1: ncol <= p columns of length <= m, column norms, and the pivoted
  // QR's permutation, remaining norms and reflector; mode 0: m columns of
  // length p and the m x m rotations; column norms
  return mode ? jacobi_ld_max(m) * (size_t)p + 5 * (size_t)m
              : jacobi_ld_max(p) * (size_t)m + jacobi_ld_max(m) * (size_t)m + 2 * (size_t)m;
}
size_t jacobi_need_doubles(int p, int m, int mode) { return jacobi_need(p, m, mode); }
// longest column the kernels take (8 elements per lane of a 64-lane group)
int jacobi_max_len() { return 512; }

struct JacobiShared {
  int rotated;
  unsigned int nrot;
  int piv;
  double tau, beta;
};

// synchronisation of the NT threads working on one problem: the workgroup
// (NT = 1024) or one wavefront (NT = 64, lanes run in lockstep; the fences
// keep the compiler from moving LDS accesses across the step boundary)
template <int NT>
__device__ __forceinline__ void team_sync() {
  if (NT > 64) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

// One pair of players: the three dot products over the group's gsz lanes and,
// if the pair is not yet orthogonal, the rotation.  The EPL elements of each
// lane (rows gl + k gsz, zero-padded) stay in registers between the dot
// products and the rotation.  The branch on `live` is uniform per group.
template <int EPL>
__device__ __forceinline__ bool jacobi_pair(double* ga_, double* gb_, double* ua, double* ub, int ldu_m,
                                            bool live, int gsz, int gl, double tol2) {
  double al = 0.0, be = 0.0, ga = 0.0;
  double x[EPL], y[EPL];
  if (live) {
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
      x[k] = ga_[gl + k * gsz];
      y[k] = gb_[gl + k * gsz];
    }
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
      al += x[k] * x[k];
      be += y[k] * y[k];
      ga += x[k] * y[k];
    }
  }
  al = group_sum(al, gsz);
  be = group_sum(be, gsz);
  ga = group_sum(ga, gsz);
  if (!(live && al > 0.0 && be > 0.0 && ga * ga > tol2 * (al * be))) return false;
  // The rotation by the smaller angle theta, tan(2 theta) = q / d with
  // d = beta - alpha, q = 2 gamma (tan theta = sign(d) q / (|d| + sqrt(d^2 +
  // q^2))), from the half-angle formulas with two reciprocal square roots and
  // no division: cos 2theta = |d| / r, sin 2theta = sign(d) q / r with
  // r = sqrt(d^2 + q^2), c^2 = (1 + cos 2theta) / 2 >= 1/2 and
  // s = sin 2theta / (2 c).  This shortens the dependent chain of each round.
  const double d = be - al, qq = 2.0 * ga;
  const double r2 = d * d + qq * qq;
  if (!(r2 > 0.0)) return false;
  const double ir = rsqrt(r2);
  const double h = 0.5 + 0.5 * (fabs(d) * ir);  // c^2
  const double ic = rsqrt(h);                    // 1 / c
  const double c = h * ic, s = 0.5 * ((d >= 0.0 ? qq : -qq) * ir) * ic;
#pragma unroll
  for (int k = 0; k < EPL; ++k) {
    ga_[gl + k * gsz] = c * x[k] - s * y[k];
    gb_[gl + k * gsz] = s * x[k] + c * y[k];
  }
  if (ua) {
#pragma unroll 4
    for (int i = gl; i < ldu_m; i += gsz) {
      const double xv = ua[i], yv = ub[i];
      ua[i] = c * xv - s * yv;
      ub[i] = s * xv + c * yv;
    }
  }
  return true;
}

// the sweeps over the round-robin tournament of ncol players (columns of G,
// stride ld); returns the number of sweeps, counts this thread's rotations
template <int NT, int EPL>
__device__ __forceinline__ int jacobi_sweeps(double* G, int ld, double* U, int ldu, int m, int ncol, int coff,
                                             int gsz, double tol2, unsigned int& my_rot, JacobiShared& sh) {
  const int tid = NT > 64 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  const int mm = ncol + (ncol & 1);
  const int npairs = mm / 2, nr = mm - 1;
  const int groups = NT / gsz;
  const int g = tid / gsz, gl = tid % gsz;
  int sweeps = 0;
  for (int sweep = 0; sweep < 40 && ncol > 1; ++sweep) {
    ++sweeps;
    int rot_here = 0;
    if (NT > 64) {
      if (tid == 0) sh.rotated = 0;
      team_sync<NT>();
    }
    for (int rnd = 0; rnd < nr; ++rnd) {
      for (int pk = g; pk < npairs; pk += groups) {
        int a, b;
        if (pk == 0) {
          a = nr;
          b = rnd;
        } else {
          a = rnd + pk;
          if (a >= nr) a -= nr;
          b = rnd - pk;
          if (b < 0) b += nr;
        }
        const bool live = a < ncol && b < ncol;
        a += coff;
        b += coff;
        double* ua = U ? U + (size_t)a * ldu : nullptr;
        double* ub = U ? U + (size_t)b * ldu : nullptr;
        if (jacobi_pair<EPL>(G + (size_t)a * ld, G + (size_t)b * ld, ua, ub, m, live, gsz, gl, tol2) && gl == 0) {
          rot_here = 1;
          ++my_rot;
        }
      }
      team_sync<NT>();
    }
    int any;
    if (NT > 64) {
      if (rot_here) sh.rotated = 1;
      team_sync<NT>();
      any = sh.rotated;
      team_sync<NT>();
    } else {
      any = __any(rot_here);
    }
    if (!any) break;
  }
  return sweeps;
}

// Preconditioner of the row-rotating mode (one-sided Jacobi after a QR with
// column pivoting, as proposed by Drmac and Veselic): Householder QR of
// B = G^T (ncol x len, B(j, c) = G[c + j ld]) with the pivot of step s taken
// over the coordinates c >= s by largest remaining norm (first index on ties;
// the norms are downdated, which only steers the choice).  Afterwards player j
// (column j of G) is row j of the trapezoidal factor, zero in the coordinates
// before j, and perm[c] is the original coordinate now stored at c.  The
// players change by an orthogonal map, which the row-rotating mode never
// needs; the permutation is undone when the vectors are written.  On the
// graded factor the sweeps roughly halve.
constexpr int kJacobiQrcpMinCols = 16;

template <int NT>
__device__ __forceinline__ void jacobi_qrcp(double* G, int ld, int len, int ncol, int32_t* perm, double* cn,
                                            double* v, JacobiShared& sh) {
  // NT = 64: one wavefront computes every uniform value itself; larger teams
  // let wavefront 0 compute them and publish them through `sh`
  const int tid = NT > 64 ? (int)threadIdx.x : (int)(threadIdx.x & 63), lane = tid & 63, wave = tid >> 6;
  for (int c = tid; c < len; c += NT) {
    perm[c] = c;
    double q = 0.0;
    for (int j = 0; j < ncol; ++j) {
      const double x = G[c + (size_t)j * ld];
      q += x * x;
    }
    cn[c] = q;
  }
  team_sync<NT>();
  // GS lanes per coordinate in the reflector application (aligned groups)
  constexpr int GS = NT >= 1024 ? 8 : 2;
  const int grp = tid / GS, gl = tid % GS, ngrp = NT / GS;
  for (int s = 0; s < ncol; ++s) {
    int pv = len;
    if (NT == 64 || wave == 0) {
      double best = -1.0;
      int bi = len;
      for (int c = s + lane; c < len; c += 64) {
        const double x = cn[c];
        if (x > best) {
          best = x;
          bi = c;
        }
      }
      for (int o = 32; o >= 1; o >>= 1) {  // the same winner on every lane
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) {
          best = ob;
          bi = oi;
        }
      }
      pv = bi;
      if (NT > 64 && lane == 0) sh.piv = bi;
    }
    if (NT > 64) {
      __syncthreads();
      pv = sh.piv;
    }
    if (pv != s && pv < len) {  // swap coordinates s and pv of every player
      for (int j = tid; j < ncol; j += NT) {
        const double a = G[s + (size_t)j * ld];
        G[s + (size_t)j * ld] = G[pv + (size_t)j * ld];
        G[pv + (size_t)j * ld] = a;
      }
      if (tid == 0) {
        const int32_t t = perm[s];
        perm[s] = perm[pv];
        perm[pv] = t;
        const double q = cn[s];
        cn[s] = cn[pv];
        cn[pv] = q;
      }
    }
    team_sync<NT>();
    if (s == ncol - 1) break;  // the last player has nothing below it
    double tau = 0.0, beta = 0.0;
    if (NT == 64 || wave == 0) {  // reflector of (B(s, s), ..., B(ncol - 1, s))
      double q = 0.0;
      for (int j = s + 1 + lane; j < ncol; j += 64) {
        const double x = G[s + (size_t)j * ld];
        q += x * x;
      }
      q = group_sum(q, 64);
      const double al = G[s + (size_t)s * ld];
      double sc = 0.0;
      beta = al;
      if (q > 0.0) {
        const double nr = sqrt(al * al + q);
        beta = al >= 0.0 ? -nr : nr;
        tau = (beta - al) / beta;
        sc = 1.0 / (al - beta);
      }
      for (int j = s + 1 + lane; j < ncol; j += 64) v[j] = G[s + (size_t)j * ld] * sc;
      if (lane == 0) {
        v[s] = 1.0;
        if (NT > 64) {
          sh.tau = tau;
          sh.beta = beta;
        }
      }
    }
    team_sync<NT>();
    if (NT > 64) {
      tau = sh.tau;
      beta = sh.beta;
    }
    // coordinate s becomes (beta, 0, ..., 0) over the players s..ncol-1
    for (int j = s + tid; j < ncol; j += NT) G[s + (size_t)j * ld] = j == s ? beta : 0.0;
    // the other coordinates c > s: B(:, c) -= tau v (v^T B(:, c)); then the
    // remaining norm loses the new B(s, c)^2
    for (int c0 = s + 1; c0 < len; c0 += ngrp) {
      const int c = c0 + grp;
      const bool act = c < len;  // uniform per group
      double w = 0.0, gcs = 0.0;
      if (act) {
        gcs = G[c + (size_t)s * ld];
        if (tau != 0.0)
          for (int j = s + gl; j < ncol; j += GS) w += v[j] * G[c + (size_t)j * ld];
      }
      w = group_sum(w, GS);
      if (act) {
        const double tw = tau * w;
        if (tau != 0.0)
          for (int j = s + gl; j < ncol; j += GS) G[c + (size_t)j * ld] -= tw * v[j];
        if (gl == 0) {
          const double ncs = gcs - tw;
          cn[c] = fmax(cn[c] - ncs * ncs, 0.0);
        }
      }
    }
    team_sync<NT>();
  }
}

// one problem on the buffer G (jacobi_need doubles) by NT threads
template <int NT>
__device__ __forceinline__ void jacobi_solve(const JacobiProb& P, double* G, int s0, JacobiShared& sh) {
  const int tid = NT > 64 ? (int)threadIdx.x : (int)(threadIdx.x & 63);
  const int m = P.m, p = P.p, mode = P.mode;
  // players: ncol columns of length len in G (stride ld, zero-padded rows)
  int ncol, len, coff;
  if (mode) {
    len = m - s0;
    ncol = min(p, len);
    coff = 0;
  } else {
    len = p;
    ncol = m - s0;
    coff = s0;
  }
  const int npairs = (ncol + (ncol & 1)) / 2;
  // at most 8 elements per lane (register budget of 1024-thread groups): long
  // columns take wider lane groups, which then take several pairs in turn
  // a wavefront alone on a problem (NT = 64) takes every pair of a round at
  // once (down to one lane per pair) and up to 32 elements per lane
  constexpr int kEplCap = NT == 64 ? 32 : 8;
  int gsz = jacobi_gsz(npairs, NT, NT == 64 ? 1 : 4);
  while (gsz < 64 && max(gsz, pow2ceil(len)) > kEplCap * gsz) gsz *= 2;
  const int ld = jacobi_ld(len, gsz);
  const int ldu = jacobi_ld(m, gsz);
  const int epl = (ld - (gsz < 32 ? gsz : 0)) / gsz;  // L / gsz, a power of two
  // G holds the columns 0..(mode ? ncol : m)-1 (mode 0 stores the zero ones too)
  const int gcols = mode ? ncol : m;
  double* U = mode ? nullptr : G + (size_t)ld * gcols;
  double* nrm = mode ? G + (size_t)ld * gcols : U + (size_t)ldu * m;
  // mode 1 with the pivoted QR first (enough players)
  const bool qrcp = mode && ncol >= kJacobiQrcpMinCols;
  int32_t* perm = (int32_t*)(nrm + m);
  if (mode) {
    for (int e = tid; e < ld * ncol; e += NT) {  // G(i, j) = R'(j, i), rows >= len zero
      const int i = e % ld, j = e / ld;
      G[e] = i < len ? P.R[j + (int64_t)i * P.ldr] : 0.0;
    }
  } else {
    for (int e = tid; e < ld * m; e += NT) {
      const int i = e % ld, j = e / ld;
      G[e] = i < p ? P.R[i + (int64_t)j * P.ldr] : 0.0;
    }
    for (int e = tid; e < ldu * m; e += NT) U[e] = (e % ldu) == (e / ldu) ? 1.0 : 0.0;
  }
  team_sync<NT>();
  if (qrcp) jacobi_qrcp<NT>(G, ld, len, ncol, perm, nrm + 2 * m, nrm + 3 * m, sh);
  // rotate while |a.b| exceeds the rounding level of a dot product of length len
  const double tol = fmax(1e-15, 2.2e-16 * len), tol2 = tol * tol;
  unsigned int my_rot = 0;
  int sweeps = 0;
  if (len > 0) {
    switch (epl) {
      case 1: sweeps = jacobi_sweeps<NT, 1>(G, ld, U, ldu, m, ncol, coff, gsz, tol2, my_rot, sh); break;
      case 2: sweeps = jacobi_sweeps<NT, 2>(G, ld, U, ldu, m, ncol, coff, gsz, tol2, my_rot, sh); break;
      case 4: sweeps = jacobi_sweeps<NT, 4>(G, ld, U, ldu, m, ncol, coff, gsz, tol2, my_rot, sh); break;
      case 8: sweeps = jacobi_sweeps<NT, 8>(G, ld, U, ldu, m, ncol, coff, gsz, tol2, my_rot, sh); break;
      default:
        if constexpr (NT == 64) {
          if (epl == 16)
            sweeps = jacobi_sweeps<NT, 16>(G, ld, U, ldu, m, ncol, coff, gsz, tol2, my_rot, sh);
          else
            sweeps = jacobi_sweeps<NT, 32>(G, ld, U, ldu, m, ncol, coff, gsz, tol2, my_rot, sh);
        }
        break;
    }
  }
  if (P.work) {
    double nrot;
    if (NT > 64) {
      if (my_rot) atomicAdd(&sh.nrot, my_rot);
      team_sync<NT>();
      nrot = sh.nrot;
    } else {
      nrot = group_sum((double)my_rot, 64);
    }
    if (tid == 0) {  // 3 dot products per pair and sweep, a rotation when applied
      const double pairs = 0.5 * ncol * (ncol - 1.0);
      double f = sweeps * pairs * 6.0 * len + nrot * (6.0 * len + (mode ? 0.0 : 6.0 * m));
      if (qrcp)  // reflector applications: 4 (ncol - s) (len - s - 1) per step
        for (int q = 0; q + 1 < ncol; ++q) f += 4.0 * (ncol - q) * (len - q - 1.0);
      *P.work = f;
    }
  }
  // nc columns carry singular values: mode 0 all m (the s0 zero ones too)
  const int nc = mode ? ncol : m;
  for (int c = tid; c < nc; c += NT) {
    double s = 0.0;
    const double* gc = G + (size_t)c * ld;
    for (int i = 0; i < len; ++i) s += gc[i] * gc[i];
    nrm[c] = sqrt(s);
  }
  team_sync<NT>();
  for (int c = tid; c < nc; c += NT) {
    const double v = nrm[c];
    int pos = 0;
    for (int d = 0; d < nc; ++d) pos += (nrm[d] > v) || (nrm[d] == v && d < c);
    P.sigma[pos] = v;
    if (P.U) {
      double* uo = P.U + (int64_t)pos * P.ldu;
      if (mode) {
        const double inv = v > 0.0 ? 1.0 / v : 0.0;
        const double* gc = G + (size_t)c * ld;
        for (int i = 0; i < s0; ++i) uo[i] = 0.0;
        if (qrcp)
          for (int i = 0; i < len; ++i) uo[s0 + perm[i]] = gc[i] * inv;
        else
          for (int i = 0; i < len; ++i) uo[s0 + i] = gc[i] * inv;
      } else {
        for (int i = 0; i < m; ++i) uo[i] = U[i + (size_t)c * ldu];
      }
    }
  }
  for (int pos = nc + tid; pos < m; pos += NT) {  // mode 1: no vector beyond ncol
    P.sigma[pos] = 0.0;
    if (P.U)
      for (int i = 0; i < m; ++i) P.U[i + (int64_t)pos * P.ldu] = 0.0;
  }
  if (P.rank && tid == 0) {
    double mx = 0.0;
    for (int c = 0; c < nc; ++c) mx = fmax(mx, nrm[c]);
    const double thr = fmax(P.eps, P.rtol * mx);
    int k = 0;
    for (int c = 0; c < nc; ++c) k += nrm[c] > thr;
    *P.rank = k;
  }
}

// Medium problems (m <= kJacobiMidM) take 256 threads, larger ones 1024: a
// round is a chain of dependent LDS loads, cross-lane sums and the rotation;
// wider groups shorten the per-lane work of long columns but lengthen the
// cross-lane sums (measured: 256 threads win at m = 64, 1024 at m ~ 100).
constexpr int kJacobiMidM = 64;

template <int NT>
__global__ __launch_bounds__(NT) void jacobi_kernel(const JacobiProb* __restrict__ probs, int nprob,
                                                    double* __restrict__ scratch, size_t slot, int lds_cap) {
  __shared__ JacobiShared sh;
  for (int pi = blockIdx.x; pi < nprob; pi += gridDim.x) {
    const JacobiProb P = probs[pi];
    if (threadIdx.x == 0) sh.nrot = 0;
    const int s0 = P.skip ? min(max(*P.skip, 0), P.m) : 0;
    if (jacobi_need(P.p, P.m, P.mode) <= (size_t)lds_cap)
      jacobi_solve<NT>(P, lds_dyn, s0, sh);
    else
      jacobi_solve<NT>(P, scratch + (size_t)blockIdx.x * slot, s0, sh);
    __syncthreads();
  }
}

// small problems (at most kJacobiSmallM columns): one wavefront
// per problem, blockDim.x / 64 per workgroup, each on its own slice of `per`
// doubles of LDS.  No workgroup barriers: a round is one wavefront's work.
constexpr int kJacobiSmallM = 32;

__global__ __launch_bounds__(256) void jacobi_small_kernel(const JacobiProb* __restrict__ probs, int nprob,
                                                           int per) {
  const int wave = threadIdx.x >> 6;
  const int pi = blockIdx.x * (blockDim.x >> 6) + wave;
  if (pi >= nprob) return;  // the whole wavefront leaves; no workgroup barriers below
  const JacobiProb P = probs[pi];
  const int s0 = P.skip ? min(max(*P.skip, 0), P.m) : 0;
  JacobiShared unused;
  jacobi_solve<64>(P, lds_dyn + (size_t)wave * per, s0, unused);
}

int jacobi_mid_max_m() { return kJacobiMidM; }

void k_jacobi(const JacobiProb* probs, int n, int lds_doubles, size_t slot, double* scratch, bool wide,
              void* stream) {
  if (n <= 0) return;
  H2_REQUIRE(slot == 0 || scratch, H2_ERR_ARG, "jacobi: global scratch missing");
  const int grid = slot == 0 ? n : std::min(n, 1024);
  if (wide)
    hipLaunchKernelGGL(jacobi_kernel<1024>, dim3(grid), dim3(1024), (size_t)lds_doubles * 8, (hipStream_t)stream,
                       probs, n, scratch, slot, lds_doubles);
  else
    hipLaunchKernelGGL(jacobi_kernel<256>, dim3(grid), dim3(256), (size_t)lds_doubles * 8, (hipStream_t)stream,
                       probs, n, scratch, slot, lds_doubles);
  HIP_OK(hipGetLastError());
}

int jacobi_small_max_m() { return kJacobiSmallM; }

void k_jacobi_small(const JacobiProb* probs, int n, int per_doubles, void* stream) {
  if (n <= 0) return;
  // several problems per workgroup only when there are enough of them to
  // fill every compute unit; otherwise each problem gets a compute unit alone
  int wpb = std::min(4, lds_limit_doubles() / std::max(per_doubles, 1));
  if (n < 4 * 256) wpb = std::min(wpb, 1);
  H2_REQUIRE(wpb >= 1, H2_ERR_ARG, "jacobi: small problems too large");
  hipLaunchKernelGGL(jacobi_small_kernel, dim3((n + wpb - 1) / wpb), dim3(64 * wpb), (size_t)wpb * per_doubles * 8,
                     (hipStream_t)stream, probs, n, per_doubles);
  HIP_OK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Spectral norms of small matrices, one wavefront per matrix.  With g =
// min(rows, cols) <= 64: the g x g Gram matrix (A^T A or A A^T) is formed in
// LDS, scaled to a unit largest diagonal entry; g steps of Lanczos with full
// reorthogonalisation (classical Gram-Schmidt, twice) reduce it to a
// tridiagonal T with the same spectrum up to rounding; the largest eigenvalue
// of T is then bracketed by Sturm counts at 64 shifts per step (one per lane)
// until the bracket is a few ulps wide.  ||A||_2 = sqrt(lambda_max).  The
// Gram matrix squares the singular values, which costs nothing in the
// relative accuracy of the largest one.
// LDS per problem: Gram g^2 | Lanczos vectors by rows and by columns (2 g^2;
// the sample staging of the Gram step, chunk x g, shares this space) | w, h,
// and the diagonal and off-diagonal of T (g each).  The chunk (16, 32 or 64
// samples) is the smallest that holds the longest side of the launch's
// blocks, up to 64: short blocks then leave room for more wavefronts.
// ---------------------------------------------------------------------------
constexpr int kNorm2MaxG = 64;
int norm2_max_dim() { return kNorm2MaxG; }
static __host__ __device__ inline size_t norm2_need(int g, int chunk) {
  return (size_t)g * g + (size_t)chunk * g + 4 * (size_t)g;
}
size_t norm2_need_doubles(int g, int chunk) { return norm2_need(g, chunk); }

// sum_{k < n} a[k sa] b[k sb] over LDS operands: the loads of eight terms
// are issued together and summed into four partial sums, so a lane waits
// for one LDS round trip per eight terms rather than per term
__device__ __forceinline__ double lds_dot(const double* a, int sa, const double* b, int sb, int n) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int k = 0;
  for (; k + 8 <= n; k += 8) {
    double x[8], y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x[u] = a[(k + u) * sa];
      y[u] = b[(k + u) * sb];
    }
    s0 += x[0] * y[0];
    s1 += x[1] * y[1];
    s2 += x[2] * y[2];
    s3 += x[3] * y[3];
    s0 += x[4] * y[4];
    s1 += x[5] * y[5];
    s2 += x[6] * y[6];
    s3 += x[7] * y[7];
  }
  for (; k < n; ++k) s0 += a[k * sa] * b[k * sb];
  return (s0 + s1) + (s2 + s3);
}

__global__ __launch_bounds__(256) void norm2_kernel(const Norm2Prob* __restrict__ probs, int nprob, int per,
                                                     int cshift) {
  const int chunk = 1 << cshift;  // samples staged per step (16, 32 or 64)
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int pi = blockIdx.x * (blockDim.x >> 6) + wave;
  if (pi >= nprob) return;  // whole wavefront; no workgroup barriers below
  const Norm2Prob P = probs[pi];
  const bool tall = P.cols <= P.rows;
  const int g = tall ? P.cols : P.rows, ns = tall ? P.rows : P.cols;
  if (g <= 0) {
    if (lane == 0) *P.out = 0.0;
    return;
  }
  // the entries are scaled by a power of two (exact) that brings the largest
  // to [1/2, 1), so the Gram matrix neither overflows nor underflows
  // (global loads eight at a time: the block is read with eight loads in
  // flight per lane instead of a chain of dependent ones)
  double amax = 0.0;
  {
    const int total = P.rows * P.cols;
    for (int e0 = lane; e0 < total; e0 += 8 * 64) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 64 * u;
        v[u] = e < total ? fabs(P.A[(e % P.rows) + (int64_t)(e / P.rows) * P.lda]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) amax = fmax(amax, v[u]);
    }
  }
  for (int o = 1; o < 64; o <<= 1) amax = fmax(amax, __shfl_xor(amax, o, 64));
  if (!(amax > 0.0) || !(amax <= DBL_MAX)) {  // zero, or not finite: passed through
    if (lane == 0) *P.out = amax;
    return;
  }
  int ex;
  (void)frexp(amax, &ex);
  const double sc = ldexp(1.0, -ex);
  double* Gm = lds_dyn + (size_t)wave * per;
  double* X = Gm + g * g;  // staging of `chunk` samples (rows, or columns) x g
  double* Wv = X + chunk * g;
  double* Hv = Wv + g;
  double* Ta = Hv + g;
  double* Tb = Ta + g;

  // ---- Gram matrix, upper triangle accumulated over chunks of samples ----
  for (int e = lane; e < g * g; e += 64) Gm[e] = 0.0;
  for (int s0 = 0; s0 < ns; s0 += chunk) {
    const int cnt = min(chunk, ns - s0);
    team_sync<64>();  // the previous chunk's reads are done
    if (tall) {
      for (int e0 = lane; e0 < chunk * g; e0 += 8 * 64) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + 64 * u, sm = e & (chunk - 1), f = e >> cshift;
          v[u] = (e < chunk * g && sm < cnt) ? P.A[(s0 + sm) + (int64_t)f * P.lda] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + 64 * u, sm = e & (chunk - 1), f = e >> cshift;
          if (e < chunk * g && sm < cnt) X[sm * g + f] = sc * v[u];
        }
      }
    } else {
      for (int e0 = lane; e0 < cnt * g; e0 += 8 * 64) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + 64 * u;
          v[u] = e < cnt * g ? P.A[(e % g) + (int64_t)(s0 + e / g) * P.lda] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + 64 * u;
          if (e < cnt * g) X[e] = sc * v[u];
        }
      }
    }
    team_sync<64>();
    for (int e = lane; e < g * g; e += 64) {
      const int f1 = e % g, f2 = e / g;
      if (f1 > f2) continue;
      Gm[e] += lds_dot(X + f1, g, X + f2, g, cnt);
    }
  }
  team_sync<64>();
  // the largest diagonal entry bounds every entry (positive semidefinite);
  // the Gram matrix is divided by it, which puts lambda_max in [1, g]
  double dmax = 0.0;
  for (int i = lane; i < g; i += 64) dmax = fmax(dmax, Gm[i + i * g]);
  for (int o = 1; o < 64; o <<= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
  const double inv = 1.0 / dmax;  // dmax >= 1/4: some entry of A is at least 1/2 after scaling
  for (int e = lane; e < g * g; e += 64) {  // lower triangle from the upper, all scaled
    const int f1 = e % g, f2 = e / g;
    if (f1 > f2) Gm[e] = Gm[f2 + f1 * g] * inv;
  }
  team_sync<64>();
  for (int e = lane; e < g * g; e += 64) {
    const int f1 = e % g, f2 = e / g;
    if (f1 <= f2) Gm[e] *= inv;
  }
  team_sync<64>();

  // ---- Householder reduction of Gm to tridiagonal form T (diagonal Ta,
  //      subdiagonal Tb): g - 2 reflectors, each applied to the trailing block
  //      as A <- A - v w^T - w v^T with p = beta A v, w = p - (beta/2)(p.v) v.
  //      Backward stable, so lambda_max(T) = lambda_max(Gm) to rounding. ----
  double* Vv = Wv;
  double* Ww = Hv;
  for (int k = 0; k + 2 < g; ++k) {
    const double xi = (lane > k && lane < g) ? Gm[lane + k * g] : 0.0;  // column k below the diagonal
    const double nx2 = wave_sum(xi * xi);
    const double x0 = Gm[(k + 1) + k * g];
    if (lane == 0) Ta[k] = Gm[k + k * g];
    if (!(nx2 > 0.0)) {  // already reduced (uniform across the wavefront)
      if (lane == 0) Tb[k] = 0.0;
      continue;
    }
    const double nx = sqrt(nx2);
    const double alpha = x0 >= 0.0 ? -nx : nx;
    const double vi = lane == k + 1 ? xi - alpha : xi;
    const double beta = 1.0 / (nx2 - alpha * x0);  // 2 / (v.v)
    if (lane == 0) Tb[k] = alpha;
    if (lane < g) Vv[lane] = vi;
    team_sync<64>();
    const int L = g - k - 1;
    double pi = 0.0;
    if (lane > k && lane < g) pi = beta * lds_dot(Gm + lane + (k + 1) * g, g, Vv + k + 1, 1, L);
    const double kc = 0.5 * beta * wave_sum(pi * vi);
    if (lane < g) Ww[lane] = pi - kc * vi;
    team_sync<64>();
    for (int e0 = lane; e0 < L * L; e0 += 8 * 64) {
      double gv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 64 * u;
        const int a = k + 1 + e % L, b = k + 1 + e / L;
        gv[u] = e < L * L ? Gm[a + b * g] - (Vv[a] * Ww[b] + Ww[a] * Vv[b]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + 64 * u;
        if (e < L * L) Gm[(k + 1 + e % L) + (k + 1 + e / L) * g] = gv[u];
      }
    }
    team_sync<64>();
  }
  if (lane == 0) {
    if (g >= 2) {
      Ta[g - 2] = Gm[(g - 2) + (g - 2) * g];
      Tb[g - 2] = Gm[(g - 1) + (g - 2) * g];
    }
    Ta[g - 1] = Gm[(g - 1) + (g - 1) * g];
  }
  const int nt = g;
  team_sync<64>();

  // ---- lambda_max(T) by multisection with Sturm counts ----
  double lo = Ta[0], hi = -1.0, bmax2 = 0.0;
  for (int i = 0; i < nt; ++i) {
    const double bl = i > 0 ? fabs(Tb[i - 1]) : 0.0, br = i + 1 < nt ? fabs(Tb[i]) : 0.0;
    lo = fmax(lo, Ta[i]);            // a diagonal entry of T is a Rayleigh quotient
    hi = fmax(hi, Ta[i] + bl + br);  // Gershgorin
    bmax2 = fmax(bmax2, br * br);
  }
  hi = fmax(hi, lo);
  const double pivmin = 0x1p-1000 * fmax(1.0, bmax2);
  for (int it = 0; it < 24 && hi - lo > 0x1p-51 * hi; ++it) {
    const double wd = hi - lo;
    const double x = lo + wd * ((double)(lane + 1) * (1.0 / 65.0));
    int neg = 0;  // eigenvalues of T below x: negative pivots of T - x I
    double d = Ta[0] - x;
    if (fabs(d) < pivmin) d = -pivmin;
    neg += d < 0.0;
    for (int i = 1; i < nt; ++i) {
      d = (Ta[i] - x) - Tb[i - 1] * Tb[i - 1] / d;
      if (fabs(d) < pivmin) d = -pivmin;
      neg += d < 0.0;
    }
    const unsigned long long above = __ballot(neg == nt);  // x above every eigenvalue
    if (above) {
      const int f = __ffsll(above) - 1;
      const double nhi = lo + wd * ((double)(f + 1) * (1.0 / 65.0));
      const double nlo = f > 0 ? lo + wd * ((double)f * (1.0 / 65.0)) : lo;
      lo = nlo;
      hi = nhi;
    } else {
      lo = lo + wd * (64.0 / 65.0);
    }
  }
  if (lane == 0) *P.out = ldexp(sqrt(0.5 * (lo + hi) * dmax), ex);
}

void k_norm2(const Norm2Prob* probs, int n, int per_doubles, int chunk, void* stream) {
  if (n <= 0) return;
  H2_REQUIRE(chunk == 16 || chunk == 32 || chunk == 64, H2_ERR_ARG, "norm2: chunk must be 16, 32 or 64");
  // problems per workgroup (one wavefront each): the most wavefronts per
  // compute unit that its 160 KiB of LDS hold, more per workgroup on ties
  constexpr size_t kCuLds = 160 * 1024;
  const size_t per_bytes = (size_t)std::max(per_doubles, 1) * 8;
  int wpb = 0, best = 0;
  for (int w = 1; w <= 4; w *= 2) {
    if (w * std::max(per_doubles, 1) > lds_limit_doubles()) break;
    const int waves = w * (int)(kCuLds / (w * per_bytes));
    if (waves >= best) {
      best = waves;
      wpb = w;
    }
  }
  if (n < 4 * 256) wpb = std::min(wpb, 1);
  H2_REQUIRE(wpb >= 1, H2_ERR_ARG, "norm2: problems too large");
  const int cshift = chunk == 16 ? 4 : chunk == 32 ? 5 : 6;
  hipLaunchKernelGGL(norm2_kernel, dim3((n + wpb - 1) / wpb), dim3(64 * wpb), (size_t)wpb * per_doubles * 8,
                     (hipStream_t)stream, probs, n, per_doubles, cshift);
  HIP_OK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// batched block fill: A[i + j ld] = (i == j ? diag : 0)
// ---------------------------------------------------------------------------
__global__ void fill_kernel(const FillItem* __restrict__ items) {
  const FillItem I = items[blockIdx.y];
  const int64_t total = (int64_t)I.rows * I.cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % I.rows, j = e / I.rows;
    I.A[i + j * I.ld] = i == j ? I.diag : 0.0;
  }
}

void k_fill(const FillItem* items, int n, void* stream) {
  if (n <= 0) return;
  for (int y0 = 0; y0 < n; y0 += 65535) {
    const int ny = std::min(65535, n - y0);
    hipLaunchKernelGGL(fill_kernel, dim3(4, ny), dim3(256), 0, (hipStream_t)stream, items + y0);
    HIP_OK(hipGetLastError());
  }
}

}  // namespace h2
