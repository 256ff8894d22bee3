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

void* dev_malloc_host(size_t bytes) {
  void* p = nullptr;
  hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(H2_ERR_ALLOC, "hipHostMalloc failed");
  }
  return p;
}

void dev_free_host(void* p) {
  if (p) (void)hipHostFree(p);
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
float dev_event_ms(void* a, void* b) {
  HIP_OK(hipEventSynchronize((hipEvent_t)b));
  float ms = 0;
  HIP_OK(hipEventElapsedTime(&ms, (hipEvent_t)a, (hipEvent_t)b));
  return ms;
}

}  // namespace h2
