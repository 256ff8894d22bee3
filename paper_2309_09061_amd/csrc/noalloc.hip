// Fixed device scratch for the entry point that allocates nothing
// (h2_matvec_noalloc).  The array lives in the code object: every device the
// library runs on holds its own copy until the process ends.  Host code never
// uses the array's name as an address: the device address is resolved once
// per device with hipGetSymbolAddress when a context is created on it, and
// that address is what the kernels receive.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace h2 {

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device of the calling
// thread), resolved on the first call for that device.
char* noalloc_scratch_resolve(int device) {
  H2_REQUIRE(device >= 0 && device < kMaxDevices, H2_ERR_ARG, "device id out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      fail(H2_ERR_DEVICE, std::string("hipGetSymbolAddress of the fixed scratch failed: ") + hipGetErrorString(e));
    }
    g_scratch_ptr[device] = (char*)p;
  }
  return g_scratch_ptr[device];
}

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

void matvec_noalloc(h2_ctx* ctx, const H2Core& A, bool trans, double alpha, const double* x, double beta,
                    double* y, int nvec) {
  H2_REQUIRE(ctx->scratch_dev, H2_ERR_DEVICE, "fixed scratch not resolved for this context");
  // exact scratch of the coefficient vectors (one per cluster and side) and
  // of the result before scaling; descriptor tables larger than the staging
  // view limit take space from the remainder
  const TreeH& T = *A.ct;
  View v{&A, trans};
  const Basis& R = v.rowb();
  const Basis& Cb = v.colb();
  size_t need = round256((size_t)T.n * nvec * sizeof(double));
  for (int c = 0; c < T.ncl; ++c)
    need += round256((size_t)std::max(Cb.rank[c], 1) * nvec * sizeof(double)) +
            round256((size_t)std::max(R.rank[c], 1) * nvec * sizeof(double));
  H2_REQUIRE(need + kNoAllocTableReserve <= kNoAllocScratchBytes, H2_ERR_ARG,
             "h2_matvec_noalloc: this matrix and nvec need " + std::to_string(need) +
                 " bytes of scratch plus " + std::to_string(kNoAllocTableReserve) +
                 " for descriptor tables, more than the fixed " + std::to_string(kNoAllocScratchBytes));
  struct Fixed {
    h2_ctx* c;
    explicit Fixed(h2_ctx* c_) : c(c_) {
      c->ws.fixed = c->scratch_dev;
      c->ws.fixed_cap = kNoAllocScratchBytes;
      c->ws.fixed_used = 0;
      c->no_alloc = true;
    }
    ~Fixed() {
      c->ws.fixed = nullptr;
      c->ws.fixed_cap = c->ws.fixed_used = 0;
      c->no_alloc = false;
    }
  } fixed(ctx);
  matvec(ctx, A, trans, alpha, x, beta, y, nvec);
}

}  // namespace h2
