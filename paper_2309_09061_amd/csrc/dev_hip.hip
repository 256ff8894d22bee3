// Device layer over the HIP runtime: allocation, asynchronous copies on the
// context stream, synchronisation and events.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace h2 {

#define HIP_OK(x)                                                              \
  do {                                                                         \
    hipError_t e_ = (x);                                                       \
    if (e_ != hipSuccess) fail(H2_ERR_DEVICE, std::string(#x ": ") + hipGetErrorString(e_)); \
  } while (0)

void dev_set_device(int device) { HIP_OK(hipSetDevice(device)); }

void* dev_malloc(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 256;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(H2_ERR_ALLOC, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  return p;
}

void dev_free(void* p) {
  if (p) (void)hipFree(p);
}

// Pinned, mapped into the device address space and coherent: kernels read it
// directly (dev_pull), seeing what the host wrote before the launch.
void* dev_malloc_host(size_t bytes) {
  void* p = nullptr;
  hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocMapped | hipHostMallocCoherent);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(H2_ERR_ALLOC, "hipHostMalloc failed");
  }
  return p;
}

void dev_free_host(void* p) {
  if (p) (void)hipHostFree(p);
}

void* dev_host_view(void* host) {
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, host, 0) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return d;
}

// A plain copy kernel reading the device view of pinned host memory: the
// upload is an ordinary launch on the stream, with no runtime copy path (which
// may wait for the stream before returning).  Both ends are padded to 256
// bytes, so whole 16-byte words are copied.
__global__ void pull_kernel(uint4* __restrict__ dst, const uint4* __restrict__ src, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// The reverse direction for a few values: a kernel writes them into the
// device view of pinned host memory (visible to the host after the stream
// is synchronised).
__global__ void push_i32_kernel(int32_t* __restrict__ dst_view, const int32_t* __restrict__ src, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst_view[i] = src[i];
}

void dev_push_i32(int32_t* dst_view, const int32_t* src, int n, void* stream) {
  if (n <= 0) return;
  const int blocks = std::min((n + 255) / 256, 64);
  hipLaunchKernelGGL(push_i32_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, dst_view, src, n);
  HIP_OK(hipGetLastError());
}

void dev_pull(void* dst, const void* src_view, size_t bytes, void* stream) {
  const size_t n = (bytes + 15) / 16;
  if (n == 0) return;
  const int blocks = (int)std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(pull_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream, (uint4*)dst,
                     (const uint4*)src_view, n);
  HIP_OK(hipGetLastError());
}

void dev_h2d(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes) HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, (hipStream_t)stream));
}
void dev_d2h(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes) HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream));
}
void dev_d2d(void* dst, const void* src, size_t bytes, void* stream) {
  if (bytes) HIP_OK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream));
}
void dev_zero(void* dst, size_t bytes, void* stream) {
  if (bytes) HIP_OK(hipMemsetAsync(dst, 0, bytes, (hipStream_t)stream));
}
void dev_sync(void* stream) { HIP_OK(hipStreamSynchronize((hipStream_t)stream)); }

// a second stream for independent passes: default priority, not ordered with
// the legacy null stream (ordering is explicit through events)
void* dev_stream_create() {
  hipStream_t s;
  HIP_OK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  return (void*)s;
}
void dev_stream_destroy(void* s) {
  if (s) (void)hipStreamDestroy((hipStream_t)s);
}
void dev_stream_wait(void* stream, void* ev) {
  HIP_OK(hipStreamWaitEvent((hipStream_t)stream, (hipEvent_t)ev, 0));
}

void* dev_event_create() {
  hipEvent_t e;
  HIP_OK(hipEventCreate(&e));
  return (void*)e;
}
void dev_event_destroy(void* ev) {
  if (ev) (void)hipEventDestroy((hipEvent_t)ev);
}
void dev_event_record(void* ev, void* stream) {
  HIP_OK(hipEventRecord((hipEvent_t)ev, (hipStream_t)stream));
}
void dev_event_sync(void* ev) { HIP_OK(hipEventSynchronize((hipEvent_t)ev)); }
float dev_event_ms(void* a, void* b) {
  HIP_OK(hipEventSynchronize((hipEvent_t)b));
  float ms = 0;
  HIP_OK(hipEventElapsedTime(&ms, (hipEvent_t)a, (hipEvent_t)b));
  return ms;
}

}  // namespace h2
