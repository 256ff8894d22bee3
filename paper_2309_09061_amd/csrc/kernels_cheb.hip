// H^2-matrix construction by tensor Chebyshev interpolation (Section 2,
// Example "Integral operator"): leaf bases l_{t,nu}(x_i), transfer matrices
// l_{t,nu}(xi_{t',nu'}), couplings g(xi_{t,nu}, xi_{s,mu}) and nearfield
// entries g(x_i, x_j); plus small utility kernels (sums of squares, identity
// blocks).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace h2 {

#define HIP_OK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) fail(H2_ERR_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

// Chebyshev point j (0-based) of `order` points on [lo, hi]
__device__ inline double cheb_node(double lo, double hi, int order, int j) {
  return 0.5 * (lo + hi) + 0.5 * (hi - lo) * cos((2.0 * (j + 1) - 1.0) * M_PI / (2.0 * order));
}

// Lagrange polynomial j of the Chebyshev points on [lo, hi] at x
__device__ inline double lagrange1(double lo, double hi, int order, int j, double x) {
  const double xj = cheb_node(lo, hi, order, j);
  double v = 1.0;
  for (int q = 0; q < order; ++q)
    if (q != j) {
      const double xq = cheb_node(lo, hi, order, q);
      v *= (x - xq) / (xj - xq);
    }
  return v;
}

// derivative of Lagrange polynomial j at x, without division by x - xi:
// l_j'(x) = sum_{q != j} 1/(xi_j - xi_q) prod_{r != j, q} (x - xi_r)/(xi_j - xi_r)
__device__ inline double lagrange1_d(double lo, double hi, int order, int j, double x) {
  const double xj = cheb_node(lo, hi, order, j);
  double s = 0.0;
  for (int q = 0; q < order; ++q) {
    if (q == j) continue;
    const double xq = cheb_node(lo, hi, order, q);
    double term = 1.0 / (xj - xq);
    for (int r = 0; r < order; ++r)
      if (r != j && r != q) {
        const double xr = cheb_node(lo, hi, order, r);
        term *= (x - xr) / (xj - xr);
      }
    s += term;
  }
  return s;
}

// -<n, grad l_{c,nu}(x)>: the row basis of the double-layer kernel
__device__ inline double lagrange_t_dn(const double* lo, const double* hi, int c, int dim, int order, int nu,
                                       const double* x, const double* n) {
  int ja[3];
  for (int a = 0; a < dim; ++a) {
    ja[a] = nu % order;
    nu /= order;
  }
  double out = 0.0;
  for (int d = 0; d < dim; ++d) {
    double term = lagrange1_d(lo[c * dim + d], hi[c * dim + d], order, ja[d], x[d]);
    for (int a = 0; a < dim; ++a)
      if (a != d) term *= lagrange1(lo[c * dim + a], hi[c * dim + a], order, ja[a], x[a]);
    out -= n[d] * term;
  }
  return out;
}

// tensor Lagrange polynomial nu of cluster c at point x (dim coordinates)
__device__ inline double lagrange_t(const double* lo, const double* hi, int c, int dim, int order,
                                    int nu, const double* x) {
  double v = 1.0;
  for (int a = 0; a < dim; ++a) {
    const int ja = nu % order;
    nu /= order;
    v *= lagrange1(lo[c * dim + a], hi[c * dim + a], order, ja, x[a]);
  }
  return v;
}

__device__ inline void interp_point(const double* lo, const double* hi, int c, int dim, int order,
                                    int nu, double* out) {
  for (int a = 0; a < dim; ++a) {
    const int ja = nu % order;
    nu /= order;
    out[a] = cheb_node(lo[c * dim + a], hi[c * dim + a], order, ja);
  }
}

__device__ inline double kernel_g(int kernel, const double* x, const double* y, int dim) {
  if (kernel == H2_K_POLY2) {
    double d = 0.0;
    for (int a = 0; a < dim; ++a) d += x[a] * y[a];
    return d * d;
  }
  double s = 0.0;
  for (int a = 0; a < dim; ++a) {
    const double d = x[a] - y[a];
    s += d * d;
  }
  const double r = sqrt(s);
  switch (kernel) {
    case H2_K_LOG: return log(r);
    case H2_K_EXPNEG: return exp(-r);
    case H2_K_INV4PI: return 1.0 / (4.0 * M_PI * r);
    default: return 1.0 / r;
  }
}

// <n(x), x - y> / (4 pi |x - y|^3), the double-layer kernel
__device__ inline double kernel_dlp(const double* x, const double* y, const double* nx, int dim) {
  double s = 0.0, p = 0.0;
  for (int a = 0; a < dim; ++a) {
    const double d = x[a] - y[a];
    s += d * d;
    p += nx[a] * d;
  }
  const double r = sqrt(s);
  return p / (4.0 * M_PI * r * r * r);
}

__device__ inline double kernel_diag(int kernel, const double* x, int dim) {
  switch (kernel) {
    case H2_K_EXPNEG: return 1.0;
    case H2_K_POLY2: return kernel_g(kernel, x, x, dim);
    default: return 0.0;
  }
}

__global__ void cheb_leaf_kernel(const ChebLeaf* d, const double* pts, const double* lo,
                                 const double* hi, int dim, int order) {
  const ChebLeaf L = d[blockIdx.y];
  int k = 1;
  for (int a = 0; a < dim; ++a) k *= order;
  const int64_t total = (int64_t)L.size * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % L.size), nu = (int)(e / L.size);
    L.V[i + nu * L.ldv] = lagrange_t(lo, hi, L.c, dim, order, nu, pts + (L.off + i) * dim);
  }
}

__global__ void cheb_leaf_dn_kernel(const ChebLeaf* d, const double* pts, const double* nrm, const double* lo,
                                    const double* hi, int dim, int order) {
  const ChebLeaf L = d[blockIdx.y];
  int k = 1;
  for (int a = 0; a < dim; ++a) k *= order;
  const int64_t total = (int64_t)L.size * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % L.size), nu = (int)(e / L.size);
    L.V[i + nu * L.ldv] =
        lagrange_t_dn(lo, hi, L.c, dim, order, nu, pts + (L.off + i) * dim, nrm + (L.off + i) * dim);
  }
}

__global__ void cheb_transfer_kernel(const ChebPair* d, const double* lo, const double* hi, int dim,
                                     int order) {
  const ChebPair P = d[blockIdx.x];  // a = child, b = parent
  int k = 1;
  for (int a = 0; a < dim; ++a) k *= order;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int nup = e % k, nu = e / k;
    double xi[3];
    interp_point(lo, hi, P.a, dim, order, nup, xi);
    P.out[nup + nu * P.ld] = lagrange_t(lo, hi, P.b, dim, order, nu, xi);
  }
}

__global__ void cheb_coupling_kernel(const ChebPair* d, const double* lo, const double* hi, int dim,
                                     int order, int kernel) {
  const ChebPair P = d[blockIdx.x];  // a = row cluster, b = column cluster
  int k = 1;
  for (int a = 0; a < dim; ++a) k *= order;
  for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
    const int nu = e % k, mu = e / k;
    double x[3], y[3];
    interp_point(lo, hi, P.a, dim, order, nu, x);
    interp_point(lo, hi, P.b, dim, order, mu, y);
    P.out[nu + mu * P.ld] = kernel_g(kernel, x, y, dim);
  }
}

__global__ void nearfield_kernel(const NearBlock* d, const double* pts, const double* nrm, int dim, int kernel) {
  const NearBlock B = d[blockIdx.y];
  const int64_t total = (int64_t)B.size_t_ * B.size_s;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(e % B.size_t_), j = (int)(e / B.size_t_);
    const double* x = pts + (B.off_t + i) * dim;
    const double* y = pts + (B.off_s + j) * dim;
    double v;
    if (B.diag && i == j)
      v = kernel_diag(kernel, x, dim);
    else if (kernel == H2_K_DLP)
      v = kernel_dlp(x, y, nrm + (B.off_t + i) * dim, dim);
    else
      v = kernel_g(kernel, x, y, dim);
    B.out[i + j * B.ld] = v;
  }
}

void k_cheb_leaf(const ChebLeaf* d, int n, const double* pts, const double* lo, const double* hi,
                 int dim, int order, void* stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cheb_leaf_kernel, dim3(8, n), dim3(256), 0, (hipStream_t)stream, d, pts, lo, hi,
                     dim, order);
  HIP_OK(hipGetLastError());
}

void k_cheb_leaf_dn(const ChebLeaf* d, int n, const double* pts, const double* nrm, const double* lo,
                    const double* hi, int dim, int order, void* stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cheb_leaf_dn_kernel, dim3(8, n), dim3(256), 0, (hipStream_t)stream, d, pts, nrm, lo, hi,
                     dim, order);
  HIP_OK(hipGetLastError());
}

void k_cheb_transfer(const ChebPair* d, int n, const double* lo, const double* hi, int dim,
                     int order, void* stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cheb_transfer_kernel, dim3(n), dim3(256), 0, (hipStream_t)stream, d, lo, hi, dim,
                     order);
  HIP_OK(hipGetLastError());
}

void k_cheb_coupling(const ChebPair* d, int n, const double* lo, const double* hi, int dim,
                     int order, int kernel, void* stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(cheb_coupling_kernel, dim3(n), dim3(256), 0, (hipStream_t)stream, d, lo, hi, dim,
                     order, kernel);
  HIP_OK(hipGetLastError());
}

void k_nearfield(const NearBlock* d, int n, const double* pts, const double* nrm, int dim, int kernel,
                 void* stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(nearfield_kernel, dim3(8, n), dim3(256), 0, (hipStream_t)stream, d, pts, nrm, dim,
                     kernel);
  HIP_OK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// utilities
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sumsq_kernel(const SumsqItem* items, const int32_t* seg_ptr,
                                                    double* out, int mode) {
  __shared__ double red[4];
  const int sg = blockIdx.x, tid = threadIdx.x;
  double s = 0.0;
  for (int it = seg_ptr[sg]; it < seg_ptr[sg + 1]; ++it) {
    const SumsqItem I = items[it];
    const int64_t total = (int64_t)I.rows * I.cols;
    for (int64_t e = tid; e < total; e += 256) {
      const double x = I.M[(e % I.rows) + (e / I.rows) * I.ld];
      s += x * x;
    }
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((tid & 63) == 0) red[tid >> 6] = s;
  __syncthreads();
  if (tid == 0) {
    const double t = red[0] + red[1] + red[2] + red[3];
    out[sg] = mode == 1 ? (t > 0.0 ? 1.0 / sqrt(t) : 0.0) : t;
  }
}

// one workgroup per group: the group's largest value, then the values at
// most rtol times it set to 0 (every read precedes every write)
__global__ __launch_bounds__(256) void drop_small_kernel(double* const* vals, const int32_t* gptr, double rtol) {
  __shared__ double red[4];
  const int g = blockIdx.x, tid = threadIdx.x;
  const int i0 = gptr[g], i1 = gptr[g + 1];
  double m = 0.0;
  for (int i = i0 + tid; i < i1; i += 256) m = fmax(m, *vals[i]);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = m;
  __syncthreads();
  const double floor = rtol * fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  for (int i = i0 + tid; i < i1; i += 256)
    if (*vals[i] <= floor) *vals[i] = 0.0;
}

void k_drop_small(double* const* vals, const int32_t* gptr, int ngroups, double rtol, void* stream) {
  if (ngroups <= 0) return;
  hipLaunchKernelGGL(drop_small_kernel, dim3(ngroups), dim3(256), 0, (hipStream_t)stream, vals, gptr, rtol);
  HIP_OK(hipGetLastError());
}

void k_sumsq(const SumsqItem* items, const int32_t* seg_ptr, int nseg, double* out, int mode,
             void* stream) {
  if (nseg <= 0) return;
  hipLaunchKernelGGL(sumsq_kernel, dim3(nseg), dim3(256), 0, (hipStream_t)stream, items, seg_ptr, out,
                     mode);
  HIP_OK(hipGetLastError());
}

}  // namespace h2

namespace h2 {

__global__ void axpby_kernel(int64_t rows, int64_t cols, double alpha, const double* x, int64_t ldx,
                             double beta, double* y, int64_t ldy) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, j = e / rows;
    const double xv = alpha * x[i + j * ldx];
    y[i + j * ldy] = beta == 0.0 ? xv : xv + beta * y[i + j * ldy];
  }
}

void k_axpby(int64_t rows, int64_t cols, double alpha, const double* x, int64_t ldx, double beta,
             double* y, int64_t ldy, void* stream) {
  if (rows <= 0 || cols <= 0) return;
  int64_t blocks = std::min<int64_t>((rows * cols + 255) / 256, 4096);
  hipLaunchKernelGGL(axpby_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, rows, cols,
                     alpha, x, ldx, beta, y, ldy);
  HIP_OK(hipGetLastError());
}

}  // namespace h2
