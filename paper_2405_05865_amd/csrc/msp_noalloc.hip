// msp_sketch_noalloc: msp_sketch for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation). The bucket
// lists and sort scratch of the sketch live in a fixed device array of this library
// instead of a caller workspace; the kernels are msp_sketch's.
#include <hip/hip_runtime.h>

#include <mutex>

#include "msp_internal.h"

namespace {

// One copy per GPU, held until the process ends. The name is a host-side stand-in for the
// array: kernels receive the device address from hipGetSymbolAddress, never the name.
static __device__ __align__(256) unsigned char scratch[MSP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device, looked up once per device
msp_status scratch_ptr(void** out) {
  int dev = -1;
  MSP_CHECK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return msp_fail(MSP_ERR_UNSUPPORTED, "device id %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return msp_fail_hip(e, "hipGetSymbolAddress(scratch)", __FILE__, __LINE__);
    if (!p || ((uintptr_t)p & 255)) return msp_fail(MSP_ERR_HIP, "static scratch has no aligned device address");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return MSP_OK;
}

}  // namespace

extern "C" msp_status msp_sketch_noalloc(void* stream, const void* A, msp_dtype a_t, int64_t m, int64_t n,
                                         int64_t lda, int64_t s, int32_t gamma, uint64_t seed, int32_t* S_rows,
                                         int8_t* S_signs, void* Y, msp_dtype y_t, int64_t ldy) {
  size_t need = 0;
  const msp_status q = msp_sketch_workspace(m, n, s, gamma, &need);
  if (q != MSP_OK) return q;
  if (need > (size_t)MSP_NOALLOC_SCRATCH_BYTES)
    return msp_fail(MSP_ERR_WORKSPACE,
                    "msp_sketch_noalloc: this sketch needs %zu bytes of scratch; the static scratch holds %zu "
                    "(use msp_sketch with a workspace)",
                    need, (size_t)MSP_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  const msp_status p = scratch_ptr(&ws);
  if (p != MSP_OK) return p;
  return msp_sketch(stream, A, a_t, m, n, lda, s, gamma, seed, S_rows, S_signs, Y, y_t, ldy, ws,
                    (size_t)MSP_NOALLOC_SCRATCH_BYTES);
}
