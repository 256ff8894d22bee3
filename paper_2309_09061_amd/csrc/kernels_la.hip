// Batched dense linear algebra for gfx950 (CDNA4, 64-lane wavefronts).
//
//  gemm_sum  grouped variable-size products C = beta C + sum alpha op(A) op(B)
//            on FP64 MFMA (v_mfma_f64_16x16x4f64), one wavefront per 16x16
//            output tile, the terms of one output accumulated in registers
//  tsqr      R factor of tall (or transposed wide) matrices, streamed in row
//            chunks through a stacked [R; chunk] Householder QR
//  jacobi    one-sided (Hestenes) Jacobi SVD with round-robin parallel pair
//            ordering; singular values and right singular vectors of R
//
// Working sets live in LDS when they fit in 64 KiB and otherwise in a
// per-workgroup slot of global scratch (generic addressing).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace h2 {

typedef double v4d __attribute__((ext_vector_type(4)));


#define HIP_OK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) fail(H2_ERR_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum for 256 threads (4 waves); `red` has >= 4 doubles
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = red[0] + red[1] + red[2] + red[3];
  return s;
}

// ---------------------------------------------------------------------------
// grouped GEMM on FP64 MFMA
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void gemm_sum_f64(const GemmOut* __restrict__ outs,
                                                    const GemmTerm* __restrict__ terms,
                                                    const int32_t* __restrict__ tiles, int ntiles) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tix = blockIdx.x * 4 + wave;
  if (tix >= ntiles) return;
  const int oi = tiles[3 * tix], i0 = tiles[3 * tix + 1], j0 = tiles[3 * tix + 2];
  const GemmOut o = outs[oi];
  const int r = lane & 15, q = lane >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
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
    const bool tA = T.flags & GT_TA, tB = T.flags & GT_TB, eye = T.flags & GT_BEYE;
    const int64_t sa_i = tA ? T.lda : 1, sa_l = tA ? 1 : T.lda;
    const int64_t sb_l = tB ? T.ldb : 1, sb_j = tB ? 1 : T.ldb;
    for (int l0 = 0; l0 < T.k; l0 += 4) {
      const int l = l0 + q;
      double a = 0.0, b = 0.0;
      if (ia && l < T.k) a = A[(int64_t)i * sa_i + (int64_t)l * sa_l];
      if (jb && l < T.k) b = eye ? (l == j ? 1.0 : 0.0) : B[(int64_t)l * sb_l + (int64_t)j * sb_j];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a * alpha, b, acc, 0, 0, 0);
    }
  }
  // FP64 accumulator layout (measured on gfx950): register v of lane (r, q)
  // holds D[4v + q][r]
  double* C = (double*)o.C;
  const int jc = j0 + r;
  if (jc < o.n) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ic = i0 + 4 * v + q;
      if (ic < o.m) {
        double* p = C + ic + (int64_t)jc * o.ldc;
        *p = o.beta ? *p + acc[v] : acc[v];
      }
    }
  }
}

void k_gemm_sum(const GemmOut* outs, const GemmTerm* terms, const int32_t* tiles, int ntiles,
                int prec, void* stream) {
  if (ntiles <= 0) return;
  (void)prec;
  dim3 grid((ntiles + 3) / 4);
  hipLaunchKernelGGL(gemm_sum_f64, grid, dim3(256), 0, (hipStream_t)stream, outs, terms, tiles, ntiles);
  HIP_OK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Householder QR of one m x n matrix W (ld) by a 256-thread workgroup
// ---------------------------------------------------------------------------
__device__ void householder_qr(double* W, int64_t ld, int m, int n, double* tau, double* red) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
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
      for (int c = jj + 1 + wave; c < n; c += 4) {
        double d = 0.0;
        for (int i = jj + lane; i < m; i += 64) d += (i == jj ? 1.0 : W[i + jj * ld]) * W[i + c * ld];
        d = wave_sum(d) * t;
        for (int i = jj + lane; i < m; i += 64) W[i + c * ld] -= d * (i == jj ? 1.0 : W[i + jj * ld]);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// TSQR: R of T (N x m), chunks of `ch` rows stacked under the running R
// ---------------------------------------------------------------------------
// rows per streamed chunk; the working set (m + chunk) x m is not monotone in
// m, so LDS-or-scratch is decided per problem with tsqr_need_doubles()
static __host__ __device__ inline int tsqr_chunk(int m) { return m <= 64 ? 64 : 32; }
static __host__ __device__ inline size_t tsqr_need(int m) { return (size_t)(m + tsqr_chunk(m)) * m; }
size_t tsqr_need_doubles(int m) { return tsqr_need(m); }

__global__ __launch_bounds__(256) void tsqr_kernel(const TsqrProb* __restrict__ probs, int nprob,
                                                   double* __restrict__ scratch, size_t slot) {
  extern __shared__ double smem[];
  __shared__ double red[4];
  const int tid = threadIdx.x;
  for (int pi = blockIdx.x; pi < nprob; pi += gridDim.x) {
    const TsqrProb P = probs[pi];
    const int m = P.m, N = P.N;
    const int ch = tsqr_chunk(m);
    const int rows_cap = m + ch;
    const bool in_lds = tsqr_need(m) <= (size_t)kLdsDoubles;
    double* B = in_lds ? smem : scratch + (size_t)blockIdx.x * slot;
    const int64_t ld = rows_cap;
    int rowsR = 0;
    const int zc = P.zero_cols ? *P.zero_cols : 0;
    for (int q0 = 0; q0 < N; q0 += ch) {
      const int cr = min(ch, N - q0);
      // load rows q0..q0+cr-1 of T into B[rowsR .. rowsR+cr-1]
      if (P.transA) {  // T(i, j) = A[j + i*lda], consecutive threads along j
        for (int e = tid; e < cr * m; e += 256) {
          const int j = e % m, i = e / m;
          const int64_t src = j + (int64_t)(q0 + i) * P.lda;
          B[rowsR + i + (int64_t)j * ld] =
              j < zc ? 0.0 : (P.prec ? (double)((const float*)P.A)[src] : ((const double*)P.A)[src]);
        }
      } else {
        for (int e = tid; e < cr * m; e += 256) {
          const int i = e % cr, j = e / cr;
          const int64_t src = (q0 + i) + (int64_t)j * P.lda;
          B[rowsR + i + (int64_t)j * ld] =
              j < zc ? 0.0 : (P.prec ? (double)((const float*)P.A)[src] : ((const double*)P.A)[src]);
        }
      }
      __syncthreads();
      const int rows = rowsR + cr;
      householder_qr(B, ld, rows, m, nullptr, red);
      rowsR = min(rows, m);
      // keep the upper triangle of the top rowsR rows, clear everything below
      for (int e = tid; e < rows * m; e += 256) {
        const int i = e % rows, j = e / rows;
        if (i > j || i >= rowsR) B[i + (int64_t)j * ld] = 0.0;
      }
      __syncthreads();
    }
    const int p = min(N, m);
    for (int e = tid; e < p * m; e += 256) {
      const int i = e % p, j = e / p;
      P.R[i + (int64_t)j * P.ldr] = (i <= j && i < rowsR) ? B[i + (int64_t)j * ld] : 0.0;
    }
    __syncthreads();
  }
}

void k_tsqr(const TsqrProb* probs, int n, size_t slot, double* scratch, void* stream) {
  if (n <= 0) return;
  H2_REQUIRE(slot == 0 || scratch, H2_ERR_ARG, "tsqr: global scratch missing");
  const int grid = slot == 0 ? n : std::min(n, 1024);
  const size_t lds = (size_t)kLdsDoubles * 8;
  hipLaunchKernelGGL(tsqr_kernel, dim3(grid), dim3(256), lds, (hipStream_t)stream, probs, n, scratch, slot);
  HIP_OK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// one-sided Jacobi SVD of R (p x m): columns rotated until orthogonal
// ---------------------------------------------------------------------------
size_t jacobi_scratch_doubles(int max_m) { return (size_t)2 * max_m * max_m + 2 * max_m; }

__global__ __launch_bounds__(256) void jacobi_kernel(const JacobiProb* __restrict__ probs, int nprob,
                                                     double* __restrict__ scratch, size_t slot) {
  extern __shared__ double smem[];
  __shared__ int rotated;
  const int tid = threadIdx.x;
  for (int pi = blockIdx.x; pi < nprob; pi += gridDim.x) {
    const JacobiProb P = probs[pi];
    const int m = P.m, p = P.p;
    if (m == 0) {
      if (tid == 0 && P.rank) *P.rank = 0;
      continue;
    }
    const bool in_lds = (int64_t)p * m + (int64_t)m * m + 2 * m <= kLdsDoubles;
    double* G = in_lds ? smem : scratch + (size_t)blockIdx.x * slot;
    double* U = G + (size_t)p * m;
    double* nrm = U + (size_t)m * m;
    for (int e = tid; e < p * m; e += 256) G[e] = P.R[(e % p) + (int64_t)(e / p) * P.ldr];
    for (int e = tid; e < m * m; e += 256) U[e] = (e % m) == (e / m) ? 1.0 : 0.0;
    __syncthreads();
    const int mm = m + (m & 1);          // players of the round-robin tournament
    const int npairs = mm / 2;
    const int gsz = npairs >= 64 ? 4 : (npairs >= 32 ? 8 : (npairs >= 16 ? 16 : (npairs >= 8 ? 32 : 64)));
    const int groups = 256 / gsz;
    const int g = tid / gsz, gl = tid % gsz;
    const double tol = 1e-15;
    for (int sweep = 0; sweep < 40; ++sweep) {
      if (tid == 0) rotated = 0;
      __syncthreads();
      for (int rnd = 0; rnd < mm - 1; ++rnd) {
        for (int pk = g; pk < npairs; pk += groups) {
          int a, b;
          if (pk == 0) {
            a = mm - 1;
            b = rnd;
          } else {
            a = (rnd + pk) % (mm - 1);
            b = (rnd - pk + (mm - 1)) % (mm - 1);
          }
          const bool live = a < m && b < m;
          double al = 0.0, be = 0.0, ga = 0.0;
          if (live) {
            const double* ga_ = G + (size_t)a * p;
            const double* gb_ = G + (size_t)b * p;
            for (int i = gl; i < p; i += gsz) {
              const double x = ga_[i], y = gb_[i];
              al += x * x;
              be += y * y;
              ga += x * y;
            }
          }
          // reduce within the group of gsz lanes (gsz divides 64)
          for (int o = gsz / 2; o >= 1; o >>= 1) {
            al += __shfl_xor(al, o, 64);
            be += __shfl_xor(be, o, 64);
            ga += __shfl_xor(ga, o, 64);
          }
          if (live && al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al * be)) {
            const double zeta = (be - al) / (2.0 * ga);
            const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
            double* ga_ = G + (size_t)a * p;
            double* gb_ = G + (size_t)b * p;
            for (int i = gl; i < p; i += gsz) {
              const double x = ga_[i], y = gb_[i];
              ga_[i] = c * x - s * y;
              gb_[i] = s * x + c * y;
            }
            double* ua = U + (size_t)a * m;
            double* ub = U + (size_t)b * m;
            for (int i = gl; i < m; i += gsz) {
              const double x = ua[i], y = ub[i];
              ua[i] = c * x - s * y;
              ub[i] = s * x + c * y;
            }
            if (gl == 0) rotated = 1;
          }
        }
        __syncthreads();
      }
      const int any = rotated;
      __syncthreads();
      if (!any) break;
    }
    // singular values = column norms; order descending (ties by index)
    for (int c = tid; c < m; c += 256) {
      double s = 0.0;
      for (int i = 0; i < p; ++i) s += G[i + (size_t)c * p] * G[i + (size_t)c * p];
      nrm[c] = sqrt(s);
    }
    __syncthreads();
    for (int c = tid; c < m; c += 256) {
      const double v = nrm[c];
      int pos = 0;
      for (int d = 0; d < m; ++d) pos += (nrm[d] > v) || (nrm[d] == v && d < c);
      P.sigma[pos] = v;
      if (P.U)
        for (int i = 0; i < m; ++i) P.U[i + (int64_t)pos * P.ldu] = U[i + (size_t)c * m];
    }
    if (P.rank) {
      __syncthreads();
      if (tid == 0) {
        double mx = 0.0;
        for (int c = 0; c < m; ++c) mx = fmax(mx, nrm[c]);
        const double thr = fmax(P.eps, P.rtol * mx);
        int k = 0;
        for (int c = 0; c < m; ++c) k += nrm[c] > thr;
        *P.rank = k;
      }
    }
    __syncthreads();
  }
}

void k_jacobi(const JacobiProb* probs, int n, int max_m, double* scratch, void* stream) {
  if (n <= 0) return;
  const bool lds_ok = (size_t)2 * max_m * max_m + 2 * max_m <= (size_t)kLdsDoubles;
  H2_REQUIRE(lds_ok || scratch, H2_ERR_ARG, "jacobi: global scratch missing");
  const int grid = lds_ok ? n : std::min(n, 1024);
  const size_t lds = (size_t)kLdsDoubles * 8;
  hipLaunchKernelGGL(jacobi_kernel, dim3(grid), dim3(256), lds, (hipStream_t)stream, probs, n,
                     scratch, jacobi_scratch_doubles(max_m));
  HIP_OK(hipGetLastError());
}

}  // namespace h2
