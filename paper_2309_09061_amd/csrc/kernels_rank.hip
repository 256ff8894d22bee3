// Rank of a truncated SVD under the relative-Frobenius rule (a variant of the
// paper's absolute rule on the block-scaled matrices, Section 5), computed
// after the Jacobi launch from the singular values it wrote.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace h2 {

#define HIP_OK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) fail(H2_ERR_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// Rank under the relative-Frobenius rule, after a Jacobi launch: from the
// singular values the launch wrote (descending), the number of leading ones
// kept while the Frobenius norm of the tail starting there exceeds eps times
// the total.  One thread per problem.
// ---------------------------------------------------------------------------
__global__ void rank_relf_kernel(const JacobiProb* __restrict__ probs, int nprob) {
  const int pi = blockIdx.x * blockDim.x + threadIdx.x;
  if (pi >= nprob) return;
  const JacobiProb P = probs[pi];
  if (!P.rank) return;
  double tot = 0.0;
  for (int i = P.m - 1; i >= 0; --i) tot += P.sigma[i] * P.sigma[i];
  const double thr2 = P.eps * P.eps * tot;
  double tail = 0.0;
  int k = 0;
  for (int i = P.m - 1; i >= 0; --i) {
    tail += P.sigma[i] * P.sigma[i];
    if (tail > thr2) {
      k = i + 1;
      break;
    }
  }
  *P.rank = k;
}

void k_rank_relf(const JacobiProb* probs, int n, void* stream) {
  if (n <= 0) return;
  hipLaunchKernelGGL(rank_relf_kernel, dim3((n + 63) / 64), dim3(64), 0, (hipStream_t)stream, probs, n);
  HIP_OK(hipGetLastError());
}

}  // namespace h2
